"""Measured device peaks (libnnp_peaks.so): the attainable FP32 and FP64 FMA
rates, the FP32 exponential rate, the FP32/FP64/BF16 matrix-core rates and
the streaming HBM copy bandwidth.

Each probe is launched on torch's current stream and timed with events on
that stream; the best of a few repetitions is kept.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnnp_peaks.so")
EXPORTS = ("nnp_peak_fma_f32", "nnp_peak_fma_f64", "nnp_peak_exp_f32", "nnp_peak_mfma_f32", "nnp_peak_mfma_f64",
           "nnp_peak_mfma_bf16", "nnp_peak_copy")

_lib = None


def load_library(path: str = LIB_PATH):
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2002_00054_amd.build")
    L = C.CDLL(path)
    for name in ("nnp_peak_fma_f32", "nnp_peak_fma_f64", "nnp_peak_exp_f32", "nnp_peak_mfma_f32",
                 "nnp_peak_mfma_f64", "nnp_peak_mfma_bf16"):
        f = getattr(L, name)
        f.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_void_p]
        f.restype = C.c_int
    L.nnp_peak_copy.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_int, C.c_void_p]
    L.nnp_peak_copy.restype = C.c_int
    _lib = L
    return L


def _best_ms(launch, reps: int) -> float:
    import torch

    launch()  # warm-up (code object load, clocks)
    best = float("inf")
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        launch()
        b.record()
        b.synchronize()
        best = min(best, a.elapsed_time(b))
    return best


def measure(reps: int = 5, copy_mib: int = 4096) -> dict:
    """Measured peaks: TFLOP/s (FMA = 2 operations), Texp/s and GB/s."""
    import torch

    L = load_library()
    cu = torch.cuda.get_device_properties(0).multi_processor_count
    blocks = cu * 32  # 8 waves of 64 lanes per SIMD on every CU
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    out = torch.empty(blocks * 256, dtype=torch.float64, device="cuda:0")
    res = {"compute_units": cu}

    def check(rc, name):
        if rc != 0:
            raise RuntimeError(f"{name} returned {rc}")

    iters = 1 << 14
    for name, fn, ops_per_iter, key in (
            ("nnp_peak_fma_f32", L.nnp_peak_fma_f32, 2 * 16, "fp32_fma_tflops"),
            ("nnp_peak_fma_f64", L.nnp_peak_fma_f64, 2 * 16, "fp64_fma_tflops"),
            ("nnp_peak_exp_f32", L.nnp_peak_exp_f32, 16, "fp32_exp_tops")):
        ms = _best_ms(lambda: check(fn(C.c_void_p(out.data_ptr()), blocks, iters, stream), name), reps)
        res[key] = ops_per_iter * iters * 256 * blocks / (ms * 1e-3) / 1e12
    # matrix cores: 4 waves per workgroup x 4 chains x operations per instruction
    m_iters = 1 << 12
    for name, fn, ops, key in (
            ("nnp_peak_mfma_f32", L.nnp_peak_mfma_f32, 2048, "mfma_fp32_tflops"),
            ("nnp_peak_mfma_f64", L.nnp_peak_mfma_f64, 2048, "mfma_fp64_tflops"),
            ("nnp_peak_mfma_bf16", L.nnp_peak_mfma_bf16, 16384, "mfma_bf16_tflops")):
        ms = _best_ms(lambda: check(fn(C.c_void_p(out.data_ptr()), blocks, m_iters, stream), name), reps)
        res[key] = 4 * 4 * ops * m_iters * blocks / (ms * 1e-3) / 1e12
    nbytes = copy_mib << 20
    src = torch.rand(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for blk in (cu * 8, cu * 32, cu * 128):
        ms = _best_ms(lambda: check(L.nnp_peak_copy(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()),
                                                    nbytes, blk, stream), "nnp_peak_copy"), reps)
        res[f"copy_gbps_{blk}_blocks"] = 2 * nbytes / (ms * 1e-3) / 1e9
    if not torch.equal(src, dst):
        raise RuntimeError("nnp_peak_copy: destination differs from source")
    ms = _best_ms(lambda: dst.copy_(src), reps)
    res["copy_gbps_torch"] = 2 * nbytes / (ms * 1e-3) / 1e9
    res["copy_gbps"] = max(v for k, v in res.items() if k.endswith("_blocks"))
    del src, dst
    torch.cuda.empty_cache()
    return res
