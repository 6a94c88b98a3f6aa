"""Python binding of the gfx950 library (``libnnp.so``, C ABI in include/nnp.h).

Argument marshalling only: every step of the energy/force path and of the
weight gradient runs in the library's HIP kernels.  torch supplies device
memory and the stream.  If the library is not built this module raises on
first use; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnnp.so")

NNP_FP64, NNP_FP32, NNP_BF16_MIXED = 0, 1, 2
PRECISIONS = {"fp64": NNP_FP64, "fp32": NNP_FP32, "bf16": NNP_BF16_MIXED}
STATUS = {0: "NNP_OK", -1: "NNP_E_ARG", -2: "NNP_E_BOX", -3: "NNP_E_TYPE", -4: "NNP_E_HIP",
          -5: "NNP_E_NOMEM", -6: "NNP_E_STATE"}

#: Every symbol include/nnp.h declares.
EXPORTS = ("nnp_create", "nnp_compute", "nnp_compute_noalloc", "nnp_compute_batch", "nnp_backward", "nnp_n_params",
           "nnp_set_params",
           "nnp_get_params", "nnp_set_profiling", "nnp_last_timings", "nnp_neighbor_capacity",
           "nnp_set_neighbor_capacity", "nnp_count_work", "nnp_md_run", "nnp_set_md_skin", "nnp_md_list_builds",
           "nnp_set_parallelism", "nnp_set_list_layout", "nnp_set_pair_masks",
           "nnp_set_derivative_mode",
           "nnp_workspace_bytes",
           "nnp_destroy", "nnp_last_error")
DERIV_MODES = {"recompute": 0, "stored": 1}
LIST_LAYOUTS = {"padded": 0, "index": 1, "compact": 2}
PARALLELISM = {"auto": 0, "wave": 1, "thread": 2, "wave2": 3}


class NNPError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class _SF(C.Structure):
    _fields_ = [("centre", C.c_int), ("kind", C.c_int), ("nbr", C.c_int * 2), ("eta", C.c_double),
                ("rs", C.c_double), ("zeta", C.c_double), ("lam", C.c_double), ("rc", C.c_double),
                ("shift", C.c_double), ("scale", C.c_double)]


class _Net(C.Structure):
    _fields_ = [("n_layers", C.c_int), ("sizes", C.POINTER(C.c_int)), ("W", C.POINTER(C.POINTER(C.c_double))),
                ("b", C.POINTER(C.POINTER(C.c_double))), ("activation", C.c_int)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libnnp.so and declare its signatures (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run `python -m paper_2002_00054_amd.build`")
    # torch ships its own HIP runtime (soname libamdhip64.so.7); loading torch
    # first makes the library bind to that same runtime, so that device
    # pointers and streams from torch are valid in the library's calls.
    import torch  # noqa: F401

    L = C.CDLL(path)
    vp, i64, dp = C.c_void_p, C.c_int64, C.POINTER(C.c_double)
    L.nnp_create.argtypes = [C.c_int, C.POINTER(C.c_char_p), C.c_int, C.POINTER(_SF), C.POINTER(_Net), C.c_int,
                             C.POINTER(vp)]
    L.nnp_compute.argtypes = [vp, i64, vp, vp, dp, dp, vp, vp, vp]
    L.nnp_compute_noalloc.argtypes = [vp, i64, vp, vp, dp, dp, vp, vp, vp]
    L.nnp_compute_batch.argtypes = [vp, C.c_int, C.POINTER(i64), vp, vp, dp, vp, vp, vp, vp]
    L.nnp_backward.argtypes = [vp, C.c_int, C.POINTER(i64), vp, vp, dp, vp, vp, vp, vp]
    L.nnp_n_params.argtypes = [vp]
    L.nnp_n_params.restype = i64
    L.nnp_set_params.argtypes = [vp, vp, C.c_int]
    L.nnp_get_params.argtypes = [vp, dp]
    L.nnp_set_profiling.argtypes = [vp, C.c_int]
    L.nnp_last_timings.argtypes = [vp, C.POINTER(C.c_char_p), dp, C.c_int]
    L.nnp_neighbor_capacity.argtypes = [vp]
    L.nnp_set_neighbor_capacity.argtypes = [vp, C.c_int]
    L.nnp_count_work.argtypes = [vp, i64, vp, vp, dp, C.POINTER(i64), vp]
    L.nnp_md_run.argtypes = [vp, i64, vp, vp, vp, vp, dp, dp, C.c_double, C.c_int, dp, dp, vp]
    L.nnp_set_list_layout.argtypes = [vp, C.c_int]
    L.nnp_set_pair_masks.argtypes = [vp, C.c_int]
    L.nnp_set_md_skin.argtypes = [vp, C.c_double]
    L.nnp_md_list_builds.argtypes = [vp]
    L.nnp_md_list_builds.restype = i64
    L.nnp_set_parallelism.argtypes = [vp, C.c_int]
    L.nnp_set_derivative_mode.argtypes = [vp, C.c_int]
    L.nnp_workspace_bytes.argtypes = [vp]
    L.nnp_workspace_bytes.restype = i64
    L.nnp_destroy.argtypes = [vp]
    L.nnp_destroy.restype = None
    L.nnp_last_error.argtypes = [vp]
    L.nnp_last_error.restype = C.c_char_p
    for name in ("nnp_create", "nnp_compute", "nnp_compute_noalloc", "nnp_compute_batch", "nnp_backward",
                 "nnp_set_params",
                 "nnp_get_params", "nnp_set_profiling", "nnp_set_neighbor_capacity", "nnp_last_timings",
                 "nnp_neighbor_capacity", "nnp_count_work", "nnp_md_run", "nnp_set_md_skin", "nnp_set_parallelism",
                 "nnp_set_list_layout", "nnp_set_pair_masks",
                 "nnp_set_derivative_mode"):
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _stream_ptr(stream):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


class Potential:
    """A potential living on the current HIP device.

    ``table``: SF records (``centre, kind, nbr, eta, rs, zeta, lam, rc, shift,
    scale``); ``nets``: per-element networks with ``W`` ([out, in] arrays) and
    ``b``; ``precision``: "fp64", "fp32" or "bf16".
    """

    def __init__(self, table, nets, precision: str = "fp32", elements=("H", "O")):
        L = load_library()
        self.precision = precision
        self.n_el = len(nets)
        sfs = (_SF * len(table))()
        for i, s in enumerate(table):
            sfs[i].centre = int(s.centre)
            sfs[i].kind = int(s.kind)
            sfs[i].nbr[0] = int(s.nbr[0])
            sfs[i].nbr[1] = int(s.nbr[-1])
            sfs[i].eta = float(s.eta)
            sfs[i].rs = float(s.rs)
            sfs[i].zeta = float(s.zeta)
            sfs[i].lam = float(s.lam)
            sfs[i].rc = float(s.rc)
            sfs[i].shift = float(s.shift)
            sfs[i].scale = float(s.scale)
        keep = []
        cnets = (_Net * len(nets))()
        for e, n in enumerate(nets):
            sizes = (C.c_int * (len(n.W) + 1))(*([n.W[0].shape[1]] + [w.shape[0] for w in n.W]))
            Ws = [np.ascontiguousarray(w, dtype=np.float64) for w in n.W]
            bs = [np.ascontiguousarray(b, dtype=np.float64) for b in n.b]
            Wp = (C.POINTER(C.c_double) * len(Ws))(*[w.ctypes.data_as(C.POINTER(C.c_double)) for w in Ws])
            bp = (C.POINTER(C.c_double) * len(bs))(*[b.ctypes.data_as(C.POINTER(C.c_double)) for b in bs])
            keep += [sizes, Ws, bs, Wp, bp]
            cnets[e].n_layers = len(n.W)
            cnets[e].sizes = sizes
            cnets[e].W = Wp
            cnets[e].b = bp
            cnets[e].activation = 0
        names = (C.c_char_p * self.n_el)(*[str(x).encode() for x in list(elements)[: self.n_el]])
        h = C.c_void_p()
        st = L.nnp_create(self.n_el, names, len(table), sfs, cnets, PRECISIONS[precision], C.byref(h))
        if st != 0:
            raise NNPError(st, L.nnp_last_error(None).decode())
        self._h = h
        self._L = L

    # ------------------------------------------------------------------
    def _check(self, st):
        if st != 0:
            raise NNPError(st, self._L.nnp_last_error(self._h).decode())

    @property
    def dtype(self):
        import torch

        return torch.float64 if self.precision == "fp64" else torch.float32

    @property
    def n_params(self) -> int:
        return int(self._L.nnp_n_params(self._h))

    def set_parallelism(self, mode: str):
        """SF and force passes: "auto" (default), "wave", "wave2" (two waves)
        or "thread" per centre."""
        self._check(self._L.nnp_set_parallelism(self._h, PARALLELISM[mode]))

    def set_list_layout(self, layout: str):
        """Neighbour list of the wave-level passes: "padded" (default),
        "index" (4-byte indices, positions gathered) or "compact" (no padding)."""
        self._check(self._L.nnp_set_list_layout(self._h, LIST_LAYOUTS[layout]))

    def set_pair_masks(self, on: bool):
        """Whether the SF pass records its pair tests for the force pass
        (default on; results are the same)."""
        self._check(self._L.nnp_set_pair_masks(self._h, 1 if on else 0))

    def set_derivative_mode(self, mode: str):
        """"recompute" (default) or "stored" (keep dG/dr per neighbour slot)."""
        self._check(self._L.nnp_set_derivative_mode(self._h, DERIV_MODES[mode]))

    @property
    def workspace_bytes(self) -> int:
        return int(self._L.nnp_workspace_bytes(self._h))

    def close(self):
        if getattr(self, "_h", None):
            self._L.nnp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _prep(self, pos, types):
        import torch

        if pos.dtype != self.dtype:
            raise TypeError(f"positions must be {self.dtype} for precision {self.precision}")
        if types.dtype != torch.int32:
            raise TypeError("types must be int32")
        if not (pos.is_cuda and types.is_cuda):
            raise TypeError("positions and types must be device tensors")
        return pos.contiguous(), types.contiguous()

    def compute(self, pos, types, box, atom_energy=True, forces=True, stream=None):
        """(E, E_i, F) of one structure; E is a Python float."""
        import torch

        pos, types = self._prep(pos, types)
        n = pos.shape[0]
        ei = torch.empty(n, dtype=self.dtype, device=pos.device) if atom_energy else None
        f = torch.empty((n, 3), dtype=self.dtype, device=pos.device) if forces else None
        boxa = (C.c_double * 3)(*[float(x) for x in box])
        e = C.c_double(0.0)
        self._check(self._L.nnp_compute(self._h, n, _ptr(pos), _ptr(types), boxa, C.byref(e), _ptr(ei), _ptr(f),
                                        _stream_ptr(stream)))
        return e.value, ei, f

    def compute_noalloc(self, pos, types, box, ei, f, stream=None):
        """nnp_compute into caller-allocated E_i [n] and F [n, 3] (either may be
        None), with every intermediate buffer in the library's static device
        workspace; returns E."""
        pos, types = self._prep(pos, types)
        for t in (ei, f):
            if t is not None and (t.dtype != self.dtype or not t.is_cuda or not t.is_contiguous()):
                raise TypeError("outputs must be contiguous device tensors of the positions' type")
        boxa = (C.c_double * 3)(*[float(x) for x in box])
        e = C.c_double(0.0)
        self._check(self._L.nnp_compute_noalloc(self._h, pos.shape[0], _ptr(pos), _ptr(types), boxa, C.byref(e),
                                                _ptr(ei), _ptr(f), _stream_ptr(stream)))
        return e.value

    def compute_batch(self, pos, types, offsets, boxes, stream=None):
        """(E_b [B] float64 device tensor, E_i, F) of a batch of structures."""
        import torch

        pos, types = self._prep(pos, types)
        offs = np.ascontiguousarray(offsets, dtype=np.int64)
        bx = np.ascontiguousarray(boxes, dtype=np.float64).reshape(-1, 3)
        nb = len(offs) - 1
        n = pos.shape[0]
        eb = torch.empty(nb, dtype=torch.float64, device=pos.device)
        ei = torch.empty(n, dtype=self.dtype, device=pos.device)
        f = torch.empty((n, 3), dtype=self.dtype, device=pos.device)
        self._check(self._L.nnp_compute_batch(self._h, nb, offs.ctypes.data_as(C.POINTER(C.c_int64)), _ptr(pos),
                                              _ptr(types), bx.ctypes.data_as(C.POINTER(C.c_double)), _ptr(eb),
                                              _ptr(ei), _ptr(f), _stream_ptr(stream)))
        return eb, ei, f

    def backward(self, pos, types, offsets, boxes, dL_dE=None, dL_dF=None, stream=None):
        """Gradient (float64 device tensor [n_params]) of a loss with the given
        dL/dE_b and dL/dF with respect to every network parameter."""
        import torch

        pos, types = self._prep(pos, types)
        offs = np.ascontiguousarray(offsets, dtype=np.int64)
        bx = np.ascontiguousarray(boxes, dtype=np.float64).reshape(-1, 3)
        nb = len(offs) - 1
        g = torch.empty(self.n_params, dtype=torch.float64, device=pos.device)
        if dL_dE is not None:
            dL_dE = dL_dE.to(torch.float64).contiguous()
        if dL_dF is not None:
            dL_dF = dL_dF.to(self.dtype).contiguous()
        self._check(self._L.nnp_backward(self._h, nb, offs.ctypes.data_as(C.POINTER(C.c_int64)), _ptr(pos),
                                         _ptr(types), bx.ctypes.data_as(C.POINTER(C.c_double)), _ptr(dL_dE),
                                         _ptr(dL_dF), _ptr(g), _stream_ptr(stream)))
        return g

    def md_run(self, pos, vel, types, box, masses, dt, n_steps, stream=None):
        """Velocity Verlet: advances the device tensors pos and vel in place by
        n_steps steps of dt fs (A, A/fs, amu per element); returns the forces
        at the final positions and the potential and kinetic energies (eV) of
        the initial state and after every step."""
        import torch

        pos, types = self._prep(pos, types)
        if vel.dtype != self.dtype or not vel.is_cuda or not vel.is_contiguous() or vel.shape != pos.shape:
            raise TypeError("vel must be a contiguous device tensor shaped and typed like pos")
        if not pos.is_contiguous():
            raise TypeError("pos must be contiguous (it is updated in place)")
        n = pos.shape[0]
        f = torch.empty((n, 3), dtype=self.dtype, device=pos.device)
        boxa = (C.c_double * 3)(*[float(x) for x in box])
        m = (C.c_double * self.n_el)(*[float(x) for x in masses])
        ep = np.zeros(n_steps + 1)
        ek = np.zeros(n_steps + 1)
        self._check(self._L.nnp_md_run(self._h, n, _ptr(pos), _ptr(vel), _ptr(f), _ptr(types), boxa, m, float(dt),
                                       int(n_steps), ep.ctypes.data_as(C.POINTER(C.c_double)),
                                       ek.ctypes.data_as(C.POINTER(C.c_double)), _stream_ptr(stream)))
        return f, ep, ek

    def set_md_skin(self, skin: float):
        """Verlet skin (A) of md_run: 0 rebuilds the neighbour list every step."""
        self._check(self._L.nnp_set_md_skin(self._h, float(skin)))

    @property
    def md_list_builds(self) -> int:
        """Neighbour-list builds of the last md_run."""
        return int(self._L.nnp_md_list_builds(self._h))

    def count_work(self, pos, types, box, stream=None) -> dict:
        """Neighbour entries, candidate neighbour pairs and triplet terms of
        one evaluation (for algorithmic-work accounting)."""
        pos, types = self._prep(pos, types)
        boxa = (C.c_double * 3)(*[float(x) for x in box])
        out = (C.c_int64 * 5)()
        self._check(self._L.nnp_count_work(self._h, pos.shape[0], _ptr(pos), _ptr(types), boxa, out,
                                           _stream_ptr(stream)))
        return {"pairs": int(out[0]), "candidates": int(out[1]), "triplets": int(out[2]),
                "angular_terms": int(out[3]), "radial_terms": int(out[4])}

    def set_params(self, flat):
        import torch

        if isinstance(flat, torch.Tensor) and flat.is_cuda:
            t = flat.detach().to(torch.float64).contiguous()
            self._check(self._L.nnp_set_params(self._h, _ptr(t), 1))
        else:
            a = np.ascontiguousarray(np.asarray(flat, dtype=np.float64))
            if a.size != self.n_params:
                raise ValueError("wrong parameter count")
            self._check(self._L.nnp_set_params(self._h, C.c_void_p(a.ctypes.data), 0))

    def get_params(self) -> np.ndarray:
        out = np.zeros(self.n_params)
        self._check(self._L.nnp_get_params(self._h, out.ctypes.data_as(C.POINTER(C.c_double))))
        return out

    def set_profiling(self, on: bool = True):
        self._check(self._L.nnp_set_profiling(self._h, int(on)))

    def timings(self) -> dict:
        names = (C.c_char_p * 32)()
        ms = (C.c_double * 32)()
        k = self._L.nnp_last_timings(self._h, names, ms, 32)
        out = {}
        for i in range(k):
            key = names[i].decode()
            out[key] = out.get(key, 0.0) + ms[i]
        return out

    @property
    def neighbor_capacity(self) -> int:
        return int(self._L.nnp_neighbor_capacity(self._h))

    def set_neighbor_capacity(self, cap: int):
        self._check(self._L.nnp_set_neighbor_capacity(self._h, int(cap)))


# ----------------------------------------------------------------------
# autograd
# ----------------------------------------------------------------------
def _autograd():
    import torch

    class NNPEnergy(torch.autograd.Function):
        """E(pos) of one structure; the gradient with respect to positions
        is -F (the hand-written adjoint computed with the forces)."""

        @staticmethod
        def forward(ctx, pos, pot, types, box):
            e, _, f = pot.compute(pos.detach(), types, box, atom_energy=False)
            ctx.save_for_backward(f)
            return torch.tensor(e, dtype=torch.float64, device=pos.device)

        @staticmethod
        def backward(ctx, gE):
            (f,) = ctx.saved_tensors
            return (-gE.to(f.dtype) * f, None, None, None)

    class NNPEnergyForces(torch.autograd.Function):
        """(E_b, F) of a batch as a function of the flat network parameters;
        the backward is the hand-written weight gradient of nnp_backward
        (descriptor derivatives recomputed).  The position gradient of F (a
        Hessian-vector product) is not provided."""

        @staticmethod
        def forward(ctx, params, pos, pot, types, offsets, boxes):
            pot.set_params(params)
            eb, _, f = pot.compute_batch(pos.detach(), types, offsets, boxes)
            ctx.pot = pot
            ctx.save_for_backward(pos, types)
            ctx.offsets = offsets
            ctx.boxes = boxes
            return eb, f

        @staticmethod
        def backward(ctx, gE, gF):
            if ctx.needs_input_grad[1]:
                raise NotImplementedError("position gradients of the forces are not provided")
            pos, types = ctx.saved_tensors
            g = ctx.pot.backward(pos, types, ctx.offsets, ctx.boxes, gE, gF)
            return (g, None, None, None, None, None)

    return NNPEnergy, NNPEnergyForces


def energy(pos, pot: Potential, types, box):
    """Differentiable total energy (autograd gives -F as d/dpos)."""
    return _autograd()[0].apply(pos, pot, types, box)


def energy_forces(params, pos, pot: Potential, types, offsets, boxes):
    """Differentiable (E_b, F) of a batch with respect to the parameters."""
    return _autograd()[1].apply(params, pos, pot, types, offsets, boxes)
