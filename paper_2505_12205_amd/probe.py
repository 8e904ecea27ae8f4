"""ctypes binding of libprobe.so (include/probe.h): hand-written streaming
kernels that measure the practical HBM ceiling (copy, non-temporal copy,
read, the fused step's in-place access pattern over 38 arrays of FP32 or
of 16-bit values at one or two per lane, and the phase-field pass's sum of
19 arrays).

Argument marshalling only; torch tensors provide device memory and the
stream.  Importing this module loads the library and raises if it has not
been built.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "_lib", "libprobe.so")


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2505_12205_amd.build` (hipcc, gfx950)")
    L = C.CDLL(LIB_PATH)
    L.pb_last_error.restype = C.c_char_p
    L.pb_stream.argtypes = [C.c_int, C.c_void_p, C.c_void_p, C.c_size_t, C.c_int, C.c_int, C.c_void_p,
                            C.POINTER(C.c_double)]
    return L


lib = _load()

EXPORTED = ("pb_stream", "pb_last_error")
KINDS = {"copy": 0, "copy_nt": 1, "read": 2, "soa_inplace": 3, "soa16_inplace": 4, "soa16x2_inplace": 5,
         "soa_sum19": 6}
# bytes moved per float of the buffer and pass
BYTES_PER_FLOAT = {k: (4 if k == "read" else 8) for k in KINDS}
BYTES_PER_FLOAT["soa_sum19"] = 4 + 4 / 19


def stream_ms(kind: str, src: torch.Tensor, dst: torch.Tensor | None = None, q: int = 0, reps: int = 10) -> float:
    """Mean ms per pass of one probe kernel over float32 device tensors."""
    ms = C.c_double()
    st = torch.cuda.current_stream(src.device).cuda_stream
    rc = lib.pb_stream(KINDS[kind], src.data_ptr(), dst.data_ptr() if dst is not None else None,
                       src.numel(), int(q), int(reps), st, C.byref(ms))
    if rc != 0:
        raise RuntimeError(f"bandwidth probe error {rc}: {lib.pb_last_error().decode()}")
    return ms.value


def ceilings(gib: float = 2.0, soa_gib: float = 9.5, reps: int = 10) -> dict:
    """GB/s of each probe kernel: the copies and the read on buffers of
    `gib` GiB, the in-place passes over 38 arrays of soa_gib / 38 GiB in all
    (9.5 GiB: the populations of the 256 x 1024 x 256 FP32 workload), the sum
    of 19 arrays over half of that (the phase field's populations)."""
    out = {}
    groups = ((("copy", "copy_nt", "read"), gib), (("soa_inplace", "soa16_inplace", "soa16x2_inplace"), soa_gib),
              (("soa_sum19",), soa_gib / 2))
    for kinds, size in groups:
        n = int(size * (1 << 30) // 4) // 152 * 152  # a multiple of 4, of 19 and of 38
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        if "copy" in kinds:
            b = torch.empty_like(a)
        elif "soa_sum19" in kinds:
            b = torch.empty(n // 19, dtype=torch.float32, device="cuda")
        else:
            b = None
        for kind in kinds:
            q = 19 if kind == "soa_sum19" else (38 if kind.startswith("soa") else 0)
            ms = stream_ms(kind, a, b, q=q, reps=reps)
            out[kind] = round(BYTES_PER_FLOAT[kind] * n / (ms * 1e-3) / 1e9, 1)
        del a, b
        torch.cuda.empty_cache()
    return out
