#!/usr/bin/env python
"""Throughput of the Behler-Parrinello energy+force path on one MI355X.

One step = one full evaluation of the 2,044,416-atom synthetic water box
(681,472 molecules on an 88^3 jittered lattice, 273.24 A, seed 22): wrap +
cell binning + neighbour-list rebuild + radial/angular symmetry functions +
per-element networks + dE/dG + force scatter + energy sum, through the C ABI
(nnp_compute).  Inputs are resident in HBM before timing starts.

Prints one JSON line:  metric/value (atom-steps/s of the FP32 form), the
roofline of the dominant kernel (the force pass) from HIP events recorded on
the library's stream during the timed steps and the library's own exact work
counts, the other arithmetic forms at the same size, and the FP64 CPU oracle
timed on a bounded sample of the same workload on this host.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "atom-steps/s energy+forces, 2M-atom water; FP32 vs BF16-MFMA at force RMSE"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "force_fp32_2M_traffic.json")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("k_triplet.inc", "common.h", "kernels.h"):
        with open(os.path.join(ROOT, "paper_2002_00054_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def time_form(pot, pos, types, box, steps, warmup):
    """ms per step over `steps` calls and per-stage HIP-event times (ms, mean)."""
    import torch

    for _ in range(warmup):
        pot.compute(pos, types, box, atom_energy=False)
    pot.set_profiling(True)
    stages = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        pot.compute(pos, types, box, atom_energy=False)
        for k, v in pot.timings().items():
            stages[k] = stages.get(k, 0.0) + v
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    pot.set_profiling(False)
    return 1e3 * dt / steps, {k: v / steps for k, v in stages.items()}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(table, nets, budget_s=12.0, nthreads=0, workload="water"):
    """The FP64 oracle on a 12,288-atom water box (or a 32,000-atom fcc box for
    the second workload) of the same generator and density (nthreads = 0:
    every thread OpenMP gets on this host)."""
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import oracle
    from paper_2002_00054_amd import synth

    pot = oracle.Potential(table, nets, n_el=len(nets))
    b = synth.water_box(16, 11) if workload == "water" else synth.fcc_box(20, 3)
    times = []
    t_start = time.perf_counter()
    while True:
        t0 = time.perf_counter()
        pot.compute(b.pos, b.types, b.box, use_cells=True, nthreads=nthreads)
        times.append(time.perf_counter() - t0)
        if time.perf_counter() - t_start > budget_s or len(times) >= 10:
            break
    times.sort()
    med = times[len(times) // 2]
    return {
        "value": b.n_atoms / med,
        "unit": "atom-steps/s",
        "cores": nthreads if nthreads > 0 else oracle.max_threads(),
        "kind": "oracle",
        "sample": (f"median of {len(times)} full energy+force evaluations (cell-list neighbours) of a "
                   f"12,288-atom water box (lattice side 16, seed 11; same generator, density and cutoff "
                   f"as the 2,044,416-atom workload), FP64 C++ oracle with OpenMP") if workload == "water" else
                  (f"median of {len(times)} full energy+force evaluations (cell-list neighbours) of a "
                   f"32,000-atom fcc box (20 cells per axis, seed 3; same generator and cutoff as the "
                   f"1,492,992-atom workload), FP64 C++ oracle with OpenMP"),
    }


def report(table, nets, sections=None):
    """Extra JSON lines instead of the contract line: the measured device peaks,
    every form over the size sweep, the single-element fcc workload (3.9 A
    cutoff, up to 1,492,992 atoms; narrow and wide angular SFs), the two
    levels of parallelism, the training step of the differentiation
    form (32 uneven boxes, loss = energy MSE + 0.1 force MSE, synthetic
    targets) with recomputed and with stored SF derivatives, the forward with
    each, velocity Verlet MD steps (throughput and energy drift), and the CPU
    oracle on one thread and on all threads.  `sections` (a set of the line
    names: peaks, sweep, training, ni, ni_g9, parallelism, layouts, pair_masks,
    forward_derivatives, md, cpu_baseline, cpu_oracle_full) limits the report to those lines; None
    runs them all (cpu_oracle_full, the oracle on the whole 2M-atom box, takes
    a few minutes of host time)."""
    import numpy as np
    import torch

    from paper_2002_00054_amd import peaks, synth
    from paper_2002_00054_amd.nnp import Potential, energy_forces

    dev = torch.device("cuda:0")

    def want(name):
        return sections is None or name in sections

    if want("peaks"):
        print(json.dumps({"report": "peaks", **peaks.measure()}), flush=True)
    for form in (("fp32", "fp64", "bf16") if want("sweep") else ()):
        pot = Potential(table, nets, precision=form)
        for side in (16, 32, 44, 64, 88):
            bb = synth.water_box(side, 22)
            x = torch.tensor(bb.pos, dtype=pot.dtype, device=dev)
            t = torch.tensor(bb.types, dtype=torch.int32, device=dev)
            ms, st = time_form(pot, x, t, bb.box, 10 if side < 64 else 5, 2)
            print(json.dumps({"report": "sweep", "form": form, "atoms": bb.n_atoms, "ms_per_step": ms,
                              "atom_steps_per_s": bb.n_atoms / (ms * 1e-3), "stages_ms": st}), flush=True)
            del x, t
        pot.close()
        torch.cuda.empty_cache()
    # differentiation form: one training step = forward of the batch + loss + weight gradient
    if want("training"):
        boxes = synth.training_batch()
        offs = np.cumsum([0] + [bx.n_atoms for bx in boxes])
        bxs = np.stack([bx.box for bx in boxes])
        rng = np.random.default_rng(5)
        N = torch.tensor([bx.n_atoms for bx in boxes], dtype=torch.float64, device=dev)
        Eh = torch.tensor(rng.normal(-1.5, 0.1, len(boxes)) * N.cpu().numpy(), dtype=torch.float64, device=dev)
        Fhat = rng.normal(0.0, 1.0, (int(offs[-1]), 3))
        for form, mode in (("fp32", "recompute"), ("fp32", "stored"), ("fp64", "recompute"), ("fp64", "stored")):
            pot = Potential(table, nets, precision=form)
            pot.set_derivative_mode(mode)
            pos = torch.tensor(np.concatenate([bx.pos for bx in boxes]), dtype=pot.dtype, device=dev)
            t = torch.tensor(np.concatenate([bx.types for bx in boxes]), dtype=torch.int32, device=dev)
            Fh = torch.tensor(Fhat, dtype=pot.dtype, device=dev)
            th = torch.tensor(synth.flat_params(nets), dtype=torch.float64, device=dev, requires_grad=True)

            def step():
                E, F = energy_forces(th, pos, pot, t, offs, bxs)
                L = torch.mean(((E - Eh) / N) ** 2) + 0.1 * torch.sum((F - Fh).double() ** 2) / (3 * N.sum())
                (g,) = torch.autograd.grad(L, th)
                return g

            for _ in range(2):
                step()
            torch.cuda.synchronize()
            # host clock per step; the median, since a step of ~30k atoms is short enough for a
            # host-side stall to dominate a mean
            ts = []
            for _ in range(10):
                t0 = time.perf_counter()
                step()
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            print(json.dumps({"report": "training", "form": form, "derivatives": mode, "boxes": len(boxes),
                              "atoms": int(offs[-1]), "ms_per_step": float(np.median(ts)) * 1e3,
                              "ms_mean": float(np.mean(ts)) * 1e3, "workspace_gb": pot.workspace_bytes / 1e9}),
                  flush=True)
            pot.close()
            torch.cuda.empty_cache()
    # second workload: single-element fcc metal, 3.9 A cutoff (the paper's Ni runs: ~1.5M atoms)
    from paper_2002_00054_amd import opcount

    ni_table, ni_nets = synth.ni_table_scaled(), synth.ni_nets()
    for form in (("fp32", "fp64", "bf16") if want("ni") else ()):
        pot = Potential(ni_table, ni_nets, precision=form, elements=("Ni",))
        for side in ((20, 40, 72) if form == "fp32" else (72,)):
            bb = synth.fcc_box(side, side)
            x = torch.tensor(bb.pos, dtype=pot.dtype, device=dev)
            t = torch.tensor(bb.types, dtype=torch.int32, device=dev)
            ms, st = time_form(pot, x, t, bb.box, 10, 2)
            line = {"report": "ni", "form": form, "atoms": bb.n_atoms, "ms_per_step": ms,
                    "atom_steps_per_s": bb.n_atoms / (ms * 1e-3), "stages_ms": st}
            if form == "fp32" and side == 72:
                counts = pot.count_work(x, t, bb.box)
                line["work_counts"] = counts
                line["force_tflops"] = opcount.flops(opcount.FORCE, counts) / (st["force"] * 1e-3) / 1e12
                line["sf_tflops"] = opcount.flops(opcount.SF, counts) / (st["sf"] * 1e-3) / 1e12
            print(json.dumps(line), flush=True)
            del x, t
        pot.close()
        torch.cuda.empty_cache()
    # the fcc workload with wide angular functions G9 (thread-per-centre passes)
    g9_table = synth.ni_table_scaled(wide=True)
    bb = synth.fcc_box(72, 72) if want("ni_g9") else None
    for form in (("fp32", "fp64") if want("ni_g9") else ()):
        pot = Potential(g9_table, ni_nets, precision=form, elements=("Ni",))
        x = torch.tensor(bb.pos, dtype=pot.dtype, device=dev)
        t = torch.tensor(bb.types, dtype=torch.int32, device=dev)
        ms, st = time_form(pot, x, t, bb.box, 5, 1)
        print(json.dumps({"report": "ni_g9", "form": form, "atoms": bb.n_atoms, "ms_per_step": ms,
                          "atom_steps_per_s": bb.n_atoms / (ms * 1e-3), "stages_ms": st}), flush=True)
        pot.close()
        del x, t
        torch.cuda.empty_cache()
    # level of parallelism of the SF and force passes: a wave per centre, two waves per centre and a
    # thread per centre, on both workloads at full size and on small water boxes (192 to 98,304
    # atoms, where the number of centres, not the work per centre, limits a launch)
    par_cases = ((("ni", synth.fcc_box(72, 72), ni_table, ni_nets, ("wave", "wave2", "thread")),
                  ("water", synth.water_box(88, 22), table, nets, ("wave", "wave2", "thread")))
                 + tuple(("water", synth.water_box(sd, 100 + sd), table, nets, ("wave", "wave2"))
                         for sd in (4, 8, 16, 32))) if want("parallelism") else ()
    for wl, bb, tb, nt, modes in par_cases:
        for mode in modes:
            pot = Potential(tb, nt, precision="fp32", elements=("Ni",) if wl == "ni" else ("H", "O"))
            pot.set_parallelism(mode)
            x = torch.tensor(bb.pos, dtype=torch.float32, device=dev)
            t = torch.tensor(bb.types, dtype=torch.int32, device=dev)
            ms, st = time_form(pot, x, t, bb.box, 3 if mode == "thread" else (5 if bb.n_atoms > 10 ** 6 else 20), 2)
            print(json.dumps({"report": "parallelism", "workload": wl, "form": "fp32", "level": mode,
                              "atoms": bb.n_atoms, "ms_per_step": ms, "stages_ms": st}), flush=True)
            pot.close()
            del x, t
            torch.cuda.empty_cache()
    # neighbour-list layout of the wave-level passes (padded displacement entries, index entries
    # with a position gather, compact rows) and the pair-test masks on and off, FP32 and FP64, on
    # both workloads at full size, with the handle's workspace
    lay_cases = tuple((wl, form, "layout", v) for wl in ("water", "ni") for form in ("fp32", "fp64")
                      for v in ("padded", "index", "compact")) if want("layouts") else ()
    lay_cases += tuple((wl, form, "pair_masks", v) for wl in ("water", "ni") for form in ("fp32", "fp64")
                       for v in ("on", "off")) if want("pair_masks") else ()
    boxes = {}
    for wl, form, what, v in lay_cases:
        if wl not in boxes:
            boxes[wl] = synth.water_box(88, 22) if wl == "water" else synth.fcc_box(72, 72)
        bb = boxes[wl]
        tb, nt = (table, nets) if wl == "water" else (ni_table, ni_nets)
        pot = Potential(tb, nt, precision=form, elements=("Ni",) if wl == "ni" else ("H", "O"))
        if what == "layout":
            pot.set_list_layout(v)
        else:
            pot.set_pair_masks(v == "on")
        x = torch.tensor(bb.pos, dtype=pot.dtype, device=dev)
        t = torch.tensor(bb.types, dtype=torch.int32, device=dev)
        ms, st = time_form(pot, x, t, bb.box, 5, 2)
        print(json.dumps({"report": what, "workload": wl, "form": form, what: v, "atoms": bb.n_atoms,
                          "ms_per_step": ms, "stages_ms": st, "workspace_gb": pot.workspace_bytes / 1e9}),
              flush=True)
        pot.close()
        del x, t
        torch.cuda.empty_cache()
    # one energy+force evaluation with the stored-Jacobian forward (one eighth of the 2M box)
    bb = synth.water_box(44, 22) if want("forward_derivatives") else None
    for mode in (("recompute", "stored") if want("forward_derivatives") else ()):
        pot = Potential(table, nets, precision="fp32")
        pot.set_derivative_mode(mode)
        x = torch.tensor(bb.pos, dtype=torch.float32, device=dev)
        t = torch.tensor(bb.types, dtype=torch.int32, device=dev)
        ms, st = time_form(pot, x, t, bb.box, 5, 2)
        print(json.dumps({"report": "forward_derivatives", "form": "fp32", "derivatives": mode, "atoms": bb.n_atoms,
                          "ms_per_step": ms, "stages_ms": st, "workspace_gb": pot.workspace_bytes / 1e9}),
              flush=True)
        pot.close()
        del x, t
        torch.cuda.empty_cache()
    # MD driver: velocity Verlet steps of the 2M box (FP32) and of a 12,288-atom box (FP64)
    md_cases = ((88, 22, "fp32", 0.5, 30), (16, 12, "fp64", 0.25, 200)) if want("md") else ()
    for side, seed, form, dt, steps in md_cases:
        bb = synth.water_box(side, seed)
        pot = Potential(table, nets, precision=form)
        t = torch.tensor(bb.types, dtype=torch.int32, device=dev)
        v_init = synth.thermal_velocities(bb.types, seed=seed)
        for skin in (0.0, 0.5, 1.0, 2.0):  # 0: neighbour list rebuilt at every step
            pot.set_md_skin(skin)
            x = torch.tensor(bb.pos, dtype=pot.dtype, device=dev)
            v = torch.tensor(v_init, dtype=pot.dtype, device=dev)
            pot.md_run(x, v, t, bb.box, synth.WATER_MASSES, dt, 1)  # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, ep, ek = pot.md_run(x, v, t, bb.box, synth.WATER_MASSES, dt, steps)
            el = time.perf_counter() - t0
            et = ep + ek
            print(json.dumps({"report": "md", "form": form, "atoms": bb.n_atoms, "dt_fs": dt, "steps": steps,
                              "skin_A": skin, "list_builds": pot.md_list_builds,
                              "ms_per_step": 1e3 * el / steps, "atom_steps_per_s": bb.n_atoms * steps / el,
                              "max_abs_dE_total_per_atom": float(np.max(np.abs(et - et[0]))) / bb.n_atoms,
                              "ekin_start": float(ek[0]), "ekin_end": float(ek[-1])}), flush=True)
            del x, v
        pot.close()
        del t
        torch.cuda.empty_cache()
    if want("cpu_oracle_full"):
        # The FP64 oracle once on the whole 2,044,416-atom box (all host threads), in 8 ranges of
        # centres that each report as they finish; then every atom of the GPU forms against it.
        sys.path.insert(0, os.path.join(ROOT, "oracle"))
        import oracle

        bb = synth.water_box(88, 22)
        opot = oracle.Potential(table, nets)
        F_ref = np.zeros((bb.n_atoms, 3))
        cuts = np.linspace(0, bb.n_atoms, 9).astype(np.int64)
        ei_parts, t_all = [], 0.0
        for k in range(8):
            t0 = time.perf_counter()
            ei_parts.append(opot.compute_centres(bb.pos, bb.types, bb.box, int(cuts[k]), int(cuts[k + 1]), F_ref))
            dt = time.perf_counter() - t0
            t_all += dt
            print(json.dumps({"report": "cpu_oracle_full_progress", "range": k + 1, "of": 8,
                              "centres": int(cuts[k + 1] - cuts[k]), "s": dt}), flush=True)
        Ei_ref = np.concatenate(ei_parts)
        line = {"report": "cpu_oracle_full", "atoms": bb.n_atoms, "cores": oracle.max_threads(),
                "cpu_model": cpu_model(), "seconds": t_all, "atom_steps_per_s": bb.n_atoms / t_all,
                "E_oracle": float(np.sum(Ei_ref))}
        for form in ("fp64", "fp32"):
            pot = Potential(table, nets, precision=form)
            x = torch.tensor(bb.pos, dtype=pot.dtype, device=dev)
            t = torch.tensor(bb.types, dtype=torch.int32, device=dev)
            e, ei, f = pot.compute(x, t, bb.box)
            ei = ei.double().cpu().numpy()
            f = f.double().cpu().numpy()
            line[form] = {"max_abs_dEi": float(np.max(np.abs(ei - Ei_ref))),
                          "max_abs_dF": float(np.max(np.abs(f - F_ref))),
                          "rel_dE": float(abs(e - line["E_oracle"]) / abs(line["E_oracle"]))}
            pot.close()
            del x, t
            torch.cuda.empty_cache()
        line["note"] = ("FP32 positions are float32-rounded on the GPU only, so the FP32 differences include "
                        "that rounding; the FP64 ones are the parity of the whole box")
        print(json.dumps(line), flush=True)
    for nt in ((0, 1) if want("cpu_baseline") else ()):  # all threads first: a thread count set once stays set
        cb = cpu_baseline(table, nets, budget_s=30.0 if nt == 1 else 12.0, nthreads=nt)
        print(json.dumps({"report": "cpu_baseline", "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
                          **cb}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=("water", "ni"), default="water",
                    help="water (the benchmark) or the single-element fcc metal at 3.9 A (second workload)")
    ap.add_argument("--n-side", type=int, default=None,
                    help="lattice side (water: 3 n^3 atoms, default 88; fcc: 4 n^3 atoms, default 72)")
    ap.add_argument("--seed", type=int, default=None)
    ap.add_argument("--forms", default="fp64,bf16", help="extra forms timed beside FP32 (comma list, '' for none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--report", action="store_true",
                    help="print only the peaks / size-sweep / training / CPU report lines")
    ap.add_argument("--sections", default=None,
                    help="with --report: comma list of report lines to run (peaks, sweep, training, ni, ni_g9, "
                         "parallelism, layouts, pair_masks, forward_derivatives, md, cpu_baseline, "
                         "cpu_oracle_full); default all")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB with a plain device copy (for HBM counter calibration) and exit")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (the spatial decomposition "
              "over several GPUs is a design note, not code); use --gpus 1", file=sys.stderr, flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        x = torch.ones(args.copy_calibration * 2 ** 18, dtype=torch.float32, device="cuda:0")
        torch.cuda.synchronize()
        y = x.clone()
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": x.numel() * 4, "copy_bytes_written": y.numel() * 4}), flush=True)
        return

    from paper_2002_00054_amd import opcount, synth
    from paper_2002_00054_amd.nnp import Potential

    table, nets = synth.water_table_scaled(), synth.water_nets()
    if args.report:
        known = {"peaks", "sweep", "training", "ni", "ni_g9", "parallelism", "layouts", "pair_masks",
                 "forward_derivatives", "md", "cpu_baseline", "cpu_oracle_full"}
        sections = None if args.sections is None else {x for x in args.sections.split(",") if x}
        if sections is not None and not sections <= known:
            ap.error(f"unknown report sections {sorted(sections - known)}; known: {sorted(known)}")
        report(table, nets, sections)
        return
    water = args.workload == "water"
    if args.n_side is None:
        args.n_side = 88 if water else 72
    if args.seed is None:
        args.seed = 22 if water else args.n_side
    if water:
        b = synth.water_box(args.n_side, args.seed)
    else:
        table, nets = synth.ni_table_scaled(), synth.ni_nets()
        b = synth.fcc_box(args.n_side, args.seed)
    n = b.n_atoms
    dev = torch.device("cuda:0")
    types = torch.tensor(b.types, dtype=torch.int32, device=dev)
    pos32 = torch.tensor(b.pos, dtype=torch.float32, device=dev)
    print(f"# workload: {n} atoms, box {b.box[0]:.2f} A", file=sys.stderr, flush=True)

    pot = Potential(table, nets, precision="fp32", elements=("H", "O") if water else ("Ni",))
    ms, stages = time_form(pot, pos32, types, b.box, args.steps, args.warmup)
    print(f"# fp32: {ms:.3f} ms/step, stages {stages}", file=sys.stderr, flush=True)
    counts = pot.count_work(pos32, types, b.box)
    f_force = opcount.flops(opcount.FORCE, counts)
    f_sf = opcount.flops(opcount.SF, counts)
    force_ms = stages.get("force", float("nan"))
    sf_ms = stages.get("sf", float("nan"))
    achieved = f_force / (force_ms * 1e-3) / 1e12
    peak = opcount.PEAK_FP32_VECTOR_TFLOPS
    traffic = None
    src = kernel_source_hash()
    if water and os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as fh:
            tr = json.load(fh)
        if tr.get("source_hash") == src:
            traffic = tr.get("bytes_per_launch")

    forms = {}
    for form in [f for f in args.forms.split(",") if f]:
        p2 = Potential(table, nets, precision=form, elements=("H", "O") if water else ("Ni",))
        x = pos32 if p2.dtype == torch.float32 else torch.tensor(b.pos, dtype=p2.dtype, device=dev)
        ms2, st2 = time_form(p2, x, types, b.box, max(2, args.steps // 3), 1)
        forms[form] = {"value": n / (ms2 * 1e-3), "ms_per_step": ms2, "stages_ms": st2}
        print(f"# {form}: {ms2:.3f} ms/step", file=sys.stderr, flush=True)
        p2.close()
        del x
        torch.cuda.empty_cache()

    out = {
        "metric": METRIC if water else "atom-steps/s energy+forces, 1.5M-atom fcc metal, 3.9 A cutoff",
        "value": n / (ms * 1e-3),
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": (f"water box {n} atoms ({n // 3} H2O, lattice side {args.n_side}, "
                                f"L={b.box[0]:.2f} A, seed {args.seed}), rc 6 A, H 27 / O 30 SFs, "
                                f"nets SF-25-25-1 tanh, neighbour list rebuilt every step") if water else
                               (f"fcc box {n} atoms ({args.n_side} cells per axis, a=3.52 A, L={b.box[0]:.2f} A, "
                                f"seed {args.seed}), rc 3.9 A, 14 SFs, nets SF-25-25-1 tanh, neighbour list "
                                f"rebuilt every step"),
                   "form": "FP32 plain"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": traffic, "kernel": "k_triplet<FP32, force>",
                     "flops_per_launch": f_force, "ms_per_launch": force_ms},
        "stages_ms": stages,
        "work_counts": counts,
        "sf_kernel": {"flops_per_launch": f_sf, "ms_per_launch": sf_ms,
                      "achieved": f_sf / (sf_ms * 1e-3) / 1e12 if sf_ms == sf_ms else None},
        "forms": forms,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(table, nets, workload=args.workload)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
