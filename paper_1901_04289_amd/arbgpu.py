"""Thin ctypes binding of libarbgpu.so (argument marshalling only).

Device buffers are torch tensors (torch provides allocation and streams);
every step of the computation runs in the library's HIP kernels.  The
binding raises if the library is missing: there is no fallback.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libarbgpu.so")

OK, NOTREADY, EINVAL, ERANGE, ENOMEM, EAGAIN, EDEVICE = 0, 1, -1, -2, -3, -4, -5
APPROX, COMPLEX, REDUCE_PREC, ALGO_LIMB, ALGO_SLICED, ALGO_RNS = 0x01, 0x02, 0x04, 0x10, 0x20, 0x40
COMPLEX_4M = 0x80
CHOICE_LIMB, CHOICE_SLICES, CHOICE_RNS256, CHOICE_RNS128 = 1, 2, 3, 4
ST_OK, ST_REFINED, ST_ERANGE = 0, 1, 2

c_p = ctypes.c_void_p
c_i64 = ctypes.c_int64
c_i32 = ctypes.c_int32
c_u32 = ctypes.c_uint32


class Arr(ctypes.Structure):
    _fields_ = [("limbs", c_p), ("ld", c_i64), ("cap", c_i32), ("exp", c_p), ("nls", c_p),
                ("rad_m", c_p), ("rad_e", c_p)]


class Out(ctypes.Structure):
    _fields_ = [("limbs", c_p), ("ld", c_i64), ("cap", c_i32), ("exp", c_p), ("nls", c_p),
                ("rad_m", c_p), ("rad_e", c_p), ("status", c_p)]


class Mat(ctypes.Structure):
    _fields_ = [("re", Arr), ("im", Arr), ("rows", c_i64), ("cols", c_i64), ("off", c_i64),
                ("rs", c_i64), ("cs", c_i64)]


class OMat(ctypes.Structure):
    _fields_ = [("re", Out), ("im", Out), ("rows", c_i64), ("cols", c_i64), ("off", c_i64),
                ("rs", c_i64), ("cs", c_i64)]


class DotJob(ctypes.Structure):
    """One dot product of a batch (the arguments of arbgpu_dot by value)."""
    _fields_ = [("res", Out * 2), ("res_idx", c_i64), ("init", Arr * 2), ("init_idx", c_i64),
                ("x", Arr * 2), ("y", Arr * 2), ("xoff", c_i64), ("xstep", c_i64), ("yoff", c_i64),
                ("ystep", c_i64), ("N", c_i64), ("p", c_i64), ("flags", c_u32), ("sub", c_i32)]


JOB_DOT, JOB_MATMUL = 1, 2


class Job(ctypes.Structure):
    """One request of the serving loop (a dot or a matrix product)."""
    _fields_ = [("kind", c_i32), ("dot", DotJob), ("C", OMat), ("A", Mat), ("B", Mat), ("p", c_i64),
                ("flags", c_u32)]


class ArbgpuError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"arbgpu error {code}: {msg}")
        self.code = code


_lib = None

EXPORTS = {
    "arbgpu_init": (ctypes.c_int, [ctypes.POINTER(c_p), ctypes.c_int, ctypes.c_size_t, ctypes.c_char_p]),
    "arbgpu_destroy": (None, [c_p]),
    "arbgpu_last_error": (ctypes.c_char_p, [c_p]),
    "arbgpu_dot": (ctypes.c_int, [c_p, ctypes.POINTER(Out), c_i64, ctypes.POINTER(Arr), c_i64, ctypes.c_int,
                                  ctypes.POINTER(Arr), c_i64, c_i64, ctypes.POINTER(Arr), c_i64, c_i64,
                                  c_i64, c_i64, c_u32, c_p]),
    "arbgpu_mat_mul": (ctypes.c_int, [c_p, ctypes.POINTER(OMat), ctypes.POINTER(Mat), ctypes.POINTER(Mat),
                                      c_i64, c_u32, c_p]),
    "arbgpu_mat_mul_exact_t": (ctypes.c_int, [c_p, c_p, c_p, c_i64, c_i32, c_p, c_p, ctypes.POINTER(Mat),
                                              ctypes.POINTER(Mat), c_u32, c_p]),
    "arbgpu_mat_mul_noalloc": (ctypes.c_int, [c_p, ctypes.POINTER(OMat), ctypes.POINTER(Mat), ctypes.POINTER(Mat),
                                              c_i64, c_u32, c_p]),
    "arbgpu_tune_mat_mul": (ctypes.c_int, [c_p, ctypes.POINTER(OMat), ctypes.POINTER(Mat), ctypes.POINTER(Mat),
                                           c_i64, c_u32, c_p, ctypes.POINTER(c_i32)]),
    "arbgpu_reserve": (ctypes.c_int, [c_p, ctypes.POINTER(Mat), ctypes.POINTER(Mat), c_i64, c_u32]),
    "arbgpu_workspace_info": (ctypes.c_int, [c_p, ctypes.POINTER(c_i64), ctypes.POINTER(c_i64)]),
    "arbgpu_mat_mul_footprint": (ctypes.c_int, [c_p, ctypes.POINTER(Mat), ctypes.POINTER(Mat), c_i64, c_u32,
                                                ctypes.POINTER(ctypes.c_size_t)]),
    "arbgpu_serve_reserve": (ctypes.c_int, [c_p, ctypes.c_void_p, c_i64]),
    "arbgpu_plan_blocks": (ctypes.c_int, [c_p, ctypes.POINTER(Mat), ctypes.POINTER(Mat), c_i64, c_u32,
                                          ctypes.POINTER(c_i64), ctypes.POINTER(ctypes.c_int32), c_i64,
                                          ctypes.POINTER(c_i64), c_p]),
    "arbgpu_batch_create": (ctypes.c_int, [c_p, ctypes.POINTER(DotJob), c_i64, ctypes.POINTER(c_p)]),
    "arbgpu_batch_create_mixed": (ctypes.c_int, [c_p, ctypes.c_void_p, c_i64, ctypes.POINTER(c_p)]),
    "arbgpu_batch_launch": (ctypes.c_int, [c_p, c_p]),
    "arbgpu_batch_tune": (ctypes.c_int, [c_p, c_p]),
    "arbgpu_batch_info": (ctypes.c_int, [c_p, ctypes.POINTER(c_i64), ctypes.c_int]),
    "arbgpu_batch_destroy": (None, [c_p]),
    "arbgpu_serve_config": (ctypes.c_int, [c_p, ctypes.c_int, ctypes.c_size_t]),
    "arbgpu_submit": (ctypes.c_int, [c_p, ctypes.POINTER(Job), c_i64, ctypes.POINTER(ctypes.c_uint64)]),
    "arbgpu_poll": (ctypes.c_int, [c_p, ctypes.c_uint64, c_i64]),
    "arbgpu_ticket_times": (ctypes.c_int, [c_p, ctypes.c_uint64, ctypes.POINTER(c_i64)]),
    "arbgpu_timing": (ctypes.c_int, [c_p, ctypes.c_int]),
    "arbgpu_plan_info": (ctypes.c_int, [c_p, ctypes.POINTER(c_i64), ctypes.c_int]),
    "arbgpu_timing_read": (ctypes.c_int, [c_p, ctypes.c_char_p, ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(c_i64)]),
    "arbgpu_probe_peaks": (ctypes.c_int, [c_p, c_p, ctypes.c_size_t, c_p, ctypes.POINTER(ctypes.c_double),
                                          ctypes.c_int]),
}

PEAK_KEYS = ["int8_mfma_tops", "fp64_mfma_tflops", "hbm_copy_gbs", "hbm_read_gbs", "mad_u64_u32_gops",
             "mul_hi_u32_gops", "clock_mhz", "compute_units"]


def load(path: str = LIB_PATH):
    """Load libarbgpu.so (raises OSError when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise OSError(f"{path} is missing: build it with `python -m paper_1901_04289_amd.build`")
    lib = ctypes.CDLL(path)
    for name, (res, args) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


# ---------------------------------------------------------------------------
# Device arrays (torch tensors)
# ---------------------------------------------------------------------------

def _torch():
    import torch
    return torch


@dataclass
class DeviceArray:
    """Operand array in device memory, limb planes [cap, ld]."""
    limbs: "object"
    exp: "object"
    nls: "object"
    rad_m: Optional["object"]
    rad_e: Optional["object"]

    @property
    def ld(self) -> int:
        return int(self.exp.shape[0])

    @property
    def cap(self) -> int:
        return int(self.limbs.shape[0])

    def arr(self) -> Arr:
        return Arr(self.limbs.data_ptr(), self.ld, self.cap, self.exp.data_ptr(), self.nls.data_ptr(),
                   self.rad_m.data_ptr() if self.rad_m is not None else None,
                   self.rad_e.data_ptr() if self.rad_e is not None else None)

    @staticmethod
    def from_host(ops, device="cuda") -> "DeviceArray":
        """Copy a host operand array (paper_1901_04289_amd.gen.Operands)."""
        torch = _torch()
        lim = torch.from_numpy(np.ascontiguousarray(ops.limbs).view(np.int32)).to(device)
        exp = torch.from_numpy(np.ascontiguousarray(ops.exp)).to(device)
        nls = torch.from_numpy(np.ascontiguousarray(ops.nls)).to(device)
        rm = re = None
        if ops.rad_m is not None:
            rm = torch.from_numpy(np.ascontiguousarray(ops.rad_m)).to(device)
            re = torch.from_numpy(np.ascontiguousarray(ops.rad_e)).to(device)
        return DeviceArray(lim, exp, nls, rm, re)


@dataclass
class DeviceOut:
    limbs: "object"
    exp: "object"
    nls: "object"
    rad_m: Optional["object"]
    rad_e: Optional["object"]
    status: "object"

    @property
    def ld(self) -> int:
        return int(self.exp.shape[0])

    @staticmethod
    def empty(count: int, p: int, radius: bool = True, device="cuda", cap: Optional[int] = None) -> "DeviceOut":
        torch = _torch()
        cap = cap or (p + 31) // 32
        return DeviceOut(torch.zeros((cap, count), dtype=torch.int32, device=device),
                         torch.zeros(count, dtype=torch.int32, device=device),
                         torch.zeros(count, dtype=torch.int32, device=device),
                         torch.zeros(count, dtype=torch.float64, device=device) if radius else None,
                         torch.zeros(count, dtype=torch.int32, device=device) if radius else None,
                         torch.full((count,), 255, dtype=torch.uint8, device=device))

    def out(self) -> Out:
        return Out(self.limbs.data_ptr(), self.ld, int(self.limbs.shape[0]), self.exp.data_ptr(),
                   self.nls.data_ptr(),
                   self.rad_m.data_ptr() if self.rad_m is not None else None,
                   self.rad_e.data_ptr() if self.rad_e is not None else None,
                   self.status.data_ptr())

    def to_host(self):
        """Copy back as (gen.Operands, status numpy array)."""
        from .gen import Operands
        return (Operands(self.limbs.cpu().numpy().view(np.uint32), self.exp.cpu().numpy(),
                         self.nls.cpu().numpy(),
                         self.rad_m.cpu().numpy() if self.rad_m is not None else None,
                         self.rad_e.cpu().numpy() if self.rad_e is not None else None),
                self.status.cpu().numpy())


def _stream_handle(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Context:
    """An arbgpu context bound to one device (-1: host-only, validation only)."""

    def __init__(self, device: int = 0, hbm_budget: int = 0, tune_cache: Optional[str] = None):
        self.lib = load()
        h = c_p()
        rc = self.lib.arbgpu_init(ctypes.byref(h), device, hbm_budget,
                                  tune_cache.encode() if tune_cache else None)
        if rc != OK:
            raise ArbgpuError(rc, f"arbgpu_init(device={device}) failed")
        self.h = h
        self.device = device

    def close(self):
        if self.h:
            self.lib.arbgpu_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def last_error(self) -> str:
        return self.lib.arbgpu_last_error(self.h).decode()

    def _check(self, rc: int):
        if rc != OK:
            raise ArbgpuError(rc, self.last_error())
        return rc

    def timing(self, enable: bool = True):
        self._check(self.lib.arbgpu_timing(self.h, int(enable)))

    def plan_info(self):
        """Shape of the last scaled-integer product (dict)."""
        buf = (c_i64 * 10)()
        self._check(self.lib.arbgpu_plan_info(self.h, buf, 10))
        keys = ["slices_a", "slices_b", "partial_planes", "groups", "inner", "rows", "cols", "parts", "primes",
                "pairs"]
        return dict(zip(keys, list(buf)))

    def timing_read(self, kernel: str):
        """(total milliseconds, launches) of the recorded launches of `kernel`."""
        ms = ctypes.c_double()
        n = c_i64()
        self._check(self.lib.arbgpu_timing_read(self.h, kernel.encode(), ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def probe_peaks(self, buf, stream=None):
        """Measured machine limits (dict keyed by PEAK_KEYS); `buf` is a
        device tensor of at least 264 MiB used as scratch."""
        out = (ctypes.c_double * 8)()
        self._check(self.lib.arbgpu_probe_peaks(self.h, ctypes.c_void_p(buf.data_ptr()),
                                                buf.numel() * buf.element_size(), _stream_handle(stream), out, 8))
        return dict(zip(PEAK_KEYS, list(out)))

    # -- raw entry points (ctypes structs) --------------------------------
    def dot_raw(self, res: Sequence[Out], res_idx: int, initial: Optional[Sequence[Arr]], init_idx: int,
                sub: bool, x: Sequence[Arr], xoff: int, xstep: int, y: Sequence[Arr], yoff: int,
                ystep: int, N: int, p: int, flags: int = 0, stream=None, check: bool = True) -> int:
        n = len(x)
        R = (Out * n)(*res)
        X = (Arr * n)(*x)
        Y = (Arr * n)(*y)
        I = (Arr * n)(*initial) if initial is not None else None
        rc = self.lib.arbgpu_dot(self.h, R, res_idx, I, init_idx, int(bool(sub)), X, xoff, xstep, Y, yoff,
                                 ystep, N, p, flags, _stream_handle(stream) if self.device >= 0 else None)
        return self._check(rc) if check else rc

    def mat_mul_raw(self, C: OMat, A: Mat, B: Mat, p: int, flags: int = 0, stream=None,
                    check: bool = True) -> int:
        rc = self.lib.arbgpu_mat_mul(self.h, ctypes.byref(C), ctypes.byref(A), ctypes.byref(B), p, flags,
                                     _stream_handle(stream) if self.device >= 0 else None)
        return self._check(rc) if check else rc

    def mat_mul_exact_t_raw(self, T_re, T_im, ldT: int, capT: int, row_v2, col_v2, A: Mat, B: Mat,
                            flags: int = 0, stream=None, check: bool = True) -> int:
        """Exact block integer T into device tensors (int32 [capT, ldT]) and
        the line scalings into int32 tensors [rows], [cols]."""
        rc = self.lib.arbgpu_mat_mul_exact_t(self.h, ctypes.c_void_p(T_re.data_ptr()),
                                             ctypes.c_void_p(T_im.data_ptr()) if T_im is not None else None,
                                             ldT, capT, ctypes.c_void_p(row_v2.data_ptr()),
                                             ctypes.c_void_p(col_v2.data_ptr()), ctypes.byref(A),
                                             ctypes.byref(B), flags,
                                             _stream_handle(stream) if self.device >= 0 else None)
        return self._check(rc) if check else rc

    def mat_mul_noalloc_raw(self, C: OMat, A: Mat, B: Mat, p: int, flags: int = 0, stream=None,
                            check: bool = True) -> int:
        """arbgpu_mat_mul with its workspace in the library's static scratch."""
        rc = self.lib.arbgpu_mat_mul_noalloc(self.h, ctypes.byref(C), ctypes.byref(A), ctypes.byref(B), p, flags,
                                             _stream_handle(stream) if self.device >= 0 else None)
        return self._check(rc) if check else rc

    def plan_blocks_raw(self, A: Mat, B: Mat, p: int, flags: int = 0, stream=None):
        """Block partition of the inner range: list of (k0, k1, kind), kind 0
        a scaled-integer block, 1 a basecase chunk."""
        cap = max(1, A.cols // 30 + 2)
        bounds = (c_i64 * (2 * cap))()
        kinds = (ctypes.c_int32 * cap)()
        nb = c_i64()
        self._check(self.lib.arbgpu_plan_blocks(self.h, ctypes.byref(A), ctypes.byref(B), p, flags, bounds, kinds,
                                                cap, ctypes.byref(nb),
                                                _stream_handle(stream) if self.device >= 0 else None))
        n = min(nb.value, cap)
        return [(bounds[2 * i], bounds[2 * i + 1], kinds[i]) for i in range(n)]

    def tune_mat_mul_raw(self, C: OMat, A: Mat, B: Mat, p: int, flags: int = 0, stream=None) -> int:
        """Time every path of this product and record the fastest for its
        class; returns the choice (1 limb, 2 slices, 3 residues/256, 4
        residues/128)."""
        ch = c_i32()
        self._check(self.lib.arbgpu_tune_mat_mul(self.h, ctypes.byref(C), ctypes.byref(A), ctypes.byref(B), p,
                                                 flags, _stream_handle(stream), ctypes.byref(ch)))
        return ch.value

    def reserve_raw(self, A: Mat, B: Mat, p: int, flags: int = 0, check: bool = True) -> int:
        """Grow the workspace for products of this shape (no allocation later)."""
        rc = self.lib.arbgpu_reserve(self.h, ctypes.byref(A), ctypes.byref(B), p, flags)
        return self._check(rc) if check else rc

    def workspace_info(self):
        """(device allocations made, workspace bytes held) by the context
        and its serving slots."""
        n, b = c_i64(), c_i64()
        self._check(self.lib.arbgpu_workspace_info(self.h, ctypes.byref(n), ctypes.byref(b)))
        return n.value, b.value

    def alloc_count(self) -> int:
        return self.workspace_info()[0]

    def footprint_raw(self, A: Mat, B: Mat, p: int, flags: int = 0) -> int:
        """Admission footprint of a matrix product, bytes."""
        n = ctypes.c_size_t()
        self._check(self.lib.arbgpu_mat_mul_footprint(self.h, ctypes.byref(A), ctypes.byref(B), p, flags,
                                                      ctypes.byref(n)))
        return n.value

    # -- request loop ------------------------------------------------------
    def serve_config(self, slots: int = 4, budget: int = 0):
        self._check(self.lib.arbgpu_serve_config(self.h, slots, budget))

    def serve_reserve(self, jobs: Sequence[Job]):
        """Reserve every slot's workspace for the largest of these jobs."""
        arr = (Job * max(1, len(jobs)))(*jobs)
        self._check(self.lib.arbgpu_serve_reserve(self.h, ctypes.cast(arr, ctypes.c_void_p), len(jobs)))

    def submit(self, jobs: Sequence[Job], check: bool = True):
        """Queue jobs; returns their tickets (or (rc, []) with check=False)."""
        arr = (Job * max(1, len(jobs)))(*jobs)
        t = (ctypes.c_uint64 * max(1, len(jobs)))()
        rc = self.lib.arbgpu_submit(self.h, arr, len(jobs), t)
        if not check:
            return rc, list(t)[:len(jobs)] if rc == OK else []
        self._check(rc)
        return list(t)[:len(jobs)]

    def poll(self, ticket: int, timeout_us: int = 0) -> int:
        return self.lib.arbgpu_poll(self.h, ticket, timeout_us)

    def wait(self, ticket: int, timeout_s: float = 120.0):
        """Polls until done; raises on the job's error or after timeout_s."""
        import time
        end = time.monotonic() + timeout_s
        while True:
            rc = self.poll(ticket, 100000)
            if rc == OK:
                return
            if rc != NOTREADY:
                self._check(rc)
            if time.monotonic() > end:
                raise TimeoutError(f"ticket {ticket} not done after {timeout_s} s")

    def ticket_times(self, ticket: int):
        """(submit, start, end) in ns of a monotonic host clock."""
        buf = (c_i64 * 3)()
        self._check(self.lib.arbgpu_ticket_times(self.h, ticket, buf))
        return tuple(buf)

    # -- convenience -------------------------------------------------------
    def plan_blocks(self, A: DeviceArray, B: DeviceArray, M: int, N: int, K: int, p: int, flags: int = 0,
                    Ai: Optional[DeviceArray] = None, Bi: Optional[DeviceArray] = None, stream=None):
        """Partition for row-major A (M x N) times B (N x K)."""
        am = Mat(A.arr(), (Ai or A).arr(), M, N, 0, N, 1)
        bm = Mat(B.arr(), (Bi or B).arr(), N, K, 0, K, 1)
        return self.plan_blocks_raw(am, bm, p, flags, stream)

    def mat_mul(self, C: DeviceOut, A: DeviceArray, B: DeviceArray, M: int, N: int, K: int, p: int,
                flags: int = 0, Ci: Optional[DeviceOut] = None, Ai: Optional[DeviceArray] = None,
                Bi: Optional[DeviceArray] = None, stream=None) -> int:
        """Row-major C (M x K) = A (M x N) B (N x K)."""
        cplx = bool(flags & COMPLEX)
        am = Mat(A.arr(), (Ai or A).arr(), M, N, 0, N, 1)
        bm = Mat(B.arr(), (Bi or B).arr(), N, K, 0, K, 1)
        cm = OMat(C.out(), (Ci or C).out(), M, K, 0, K, 1)
        if cplx and (Ai is None or Bi is None or Ci is None):
            raise ValueError("complex product needs imaginary parts")
        return self.mat_mul_raw(cm, am, bm, p, flags, stream)


def dot_job(res: Sequence[Out], res_idx: int, x: Sequence[Arr], xoff: int, xstep: int, y: Sequence[Arr],
            yoff: int, ystep: int, N: int, p: int, flags: int = 0, initial: Optional[Sequence[Arr]] = None,
            init_idx: int = 0, sub: bool = False) -> DotJob:
    """Pack one batch job; sequences hold one part (real) or two (complex)."""
    j = DotJob()
    for q in range(len(x)):
        j.res[q] = res[q]
        j.x[q] = x[q]
        j.y[q] = y[q]
        if initial is not None:
            j.init[q] = initial[q]
    j.res_idx, j.init_idx = res_idx, init_idx
    j.xoff, j.xstep, j.yoff, j.ystep, j.N, j.p = xoff, xstep, yoff, ystep, N, p
    j.flags, j.sub = flags, int(bool(sub))
    return j


class Batch:
    """A resident batch replayed as one graph launch: dot products
    (DotJob), or dot and matrix-product requests (Job) with mixed=True."""

    def __init__(self, ctx: "Context", jobs, mixed: bool = False):
        self.ctx = ctx
        h = c_p()
        if mixed:
            arr = (Job * max(1, len(jobs)))(*jobs)
            ctx._check(ctx.lib.arbgpu_batch_create_mixed(ctx.h, ctypes.cast(arr, ctypes.c_void_p), len(jobs),
                                                         ctypes.byref(h)))
        else:
            arr = (DotJob * max(1, len(jobs)))(*jobs)
            ctx._check(ctx.lib.arbgpu_batch_create(ctx.h, arr, len(jobs), ctypes.byref(h)))
        self.h = h

    def launch(self, stream=None):
        self.ctx._check(self.ctx.lib.arbgpu_batch_launch(self.h, _stream_handle(stream)))

    def tune(self, stream=None):
        self.ctx._check(self.ctx.lib.arbgpu_batch_tune(self.h, _stream_handle(stream)))

    def info(self):
        buf = (c_i64 * 256)()
        self.ctx._check(self.ctx.lib.arbgpu_batch_info(self.h, buf, 256))
        v = list(buf)
        shapes = [dict(ns=v[3 + 5 * k], na=v[4 + 5 * k], tasks=v[5 + 5 * k], waves=v[6 + 5 * k],
                       tuned_us=v[7 + 5 * k]) for k in range(min(v[2], 50))]
        return dict(jobs=v[0], tasks=v[1], shapes=shapes)

    def close(self):
        if self.h:
            self.ctx.lib.arbgpu_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def matmul_job(C: OMat, A: Mat, B: Mat, p: int, flags: int = 0) -> Job:
    j = Job()
    j.kind = JOB_MATMUL
    j.C, j.A, j.B, j.p, j.flags = C, A, B, p, flags
    return j


def dot_request(job: DotJob) -> Job:
    j = Job()
    j.kind = JOB_DOT
    j.dot = job
    return j

