"""Python binding of libpk_probe.so (include/pk_probe.h): the atomic
throughput probes that give the pipeline's atomic rooflines their
denominators.  Argument marshalling and HIP-event timing only; every probe
runs in the library's kernels."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpk_probe.so")
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1404_6293_amd.build`")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.pkp_lds_min_u64.restype = C.c_int
        L.pkp_lds_min_u64.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, P, P]
        L.pkp_global_min_u64.restype = C.c_int
        L.pkp_global_min_u64.argtypes = [P, P, C.c_int64, P]
        L.pkp_global_add_f32.restype = C.c_int
        L.pkp_global_add_f32.argtypes = [P, P, P, C.c_int64, P]
        _lib = L
    return _lib


def _stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


def _timed(torch, fn, reps):
    """Median milliseconds of `fn` between HIP events on the current stream."""
    ts = []
    st = torch.cuda.current_stream()
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        fn()
        e1.record(st)
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    ts.sort()
    return ts[len(ts) // 2]


def _ok(name, rc):
    if rc != 0:
        raise RuntimeError(f"{name} failed (status {rc})")


def lds_min_u64_rate(tile_keys: int, with_return: bool, workgroups: int = 4096,
                     iters: int = 256, reps: int = 5) -> float:
    """64-bit LDS atomic mins per second (G/s) into per-workgroup tiles of
    `tile_keys` keys at uniform random addresses."""
    import torch
    L = lib()
    sink = torch.zeros(workgroups, dtype=torch.int64, device="cuda")
    run = lambda: _ok("pkp_lds_min_u64", L.pkp_lds_min_u64(  # noqa: E731
        int(tile_keys), int(with_return), workgroups, iters, sink.data_ptr(), _stream()))
    run()
    ms = _timed(torch, run, reps)
    return workgroups * 256 * iters / (ms * 1e-3) / 1e9


def global_min_u64_rate(addr, nkeys: int, reps: int = 5) -> float:
    """Device-scope 64-bit atomic mins per second (G/s), one per entry of the
    int32 device tensor `addr` into a buffer of `nkeys` keys (all ones before
    each run, like the depth test's cleared key buffer)."""
    import torch
    L = lib()
    keys = torch.empty(nkeys, dtype=torch.int64, device="cuda")
    m = int(addr.numel())

    def run():
        keys.fill_(-1)
        _ok("pkp_global_min_u64", L.pkp_global_min_u64(keys.data_ptr(), addr.data_ptr(), m,
                                                        _stream()))
    run()
    fill_ms = _timed(torch, lambda: keys.fill_(-1), reps)
    ms = _timed(torch, run, reps) - fill_ms
    return m / (max(ms, 1e-6) * 1e-3) / 1e9


def global_add_f32_rate(addr, nvals: int, reps: int = 5) -> float:
    """Device-scope float32 atomic adds per second (G/s), one per entry of the
    int32 device tensor `addr` into a zeroed buffer of `nvals` floats."""
    import torch
    L = lib()
    dst = torch.zeros(nvals, dtype=torch.float32, device="cuda")
    m = int(addr.numel())
    run = lambda: _ok("pkp_global_add_f32", L.pkp_global_add_f32(  # noqa: E731
        dst.data_ptr(), addr.data_ptr(), None, m, _stream()))
    run()
    ms = _timed(torch, run, reps)
    return m / (ms * 1e-3) / 1e9
