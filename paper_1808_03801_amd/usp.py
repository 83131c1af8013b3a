"""ctypes binding of libusp (include/usp.h): argument marshalling only.

Every step of the solver runs in the HIP kernels of ``libusp.so``; this module
converts a :class:`paper_1808_03801_amd.problems.Problem` into the C structs,
hands PyTorch's caching allocator and current stream to the library, and
copies states in and out.  It raises if the library or the GPU is missing:
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libusp.so")

NMOM = 13
NCS = 4 * NMOM + 2
NF = 18
NDIAG = 48

STATUS = {0: "USP_OK", -1: "USP_EINVAL", -2: "USP_ENOMEM", -3: "USP_ECAPACITY",
          -4: "USP_EWINDOW", -5: "USP_EDEVICE", -7: "USP_ESTATE", -8: "USP_ENOLIB",
          -9: "USP_ENONFINITE"}


class UspError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Gas(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("m", "kB", "mu_ref", "T_ref", "omega", "Pr")]


class Face(C.Structure):
    _fields_ = [("kind", C.c_int), ("T", C.c_double), ("u", C.c_double * 3), ("n", C.c_double),
                ("split", C.c_double), ("n_b", C.c_double), ("T_b", C.c_double)]


class ProblemC(C.Structure):
    _fields_ = [("dim", C.c_int), ("nx", C.c_int), ("ny", C.c_int)] + \
               [(n, C.c_double) for n in ("x0", "x1", "y0", "y1", "dx", "dy", "inv_dx",
                                          "inv_dy", "vcell")] + \
               [("face", Face * 4), ("accel", C.c_double * 3), ("plate", C.c_int)] + \
               [(n, C.c_double) for n in ("plate_x", "plate_ylo", "plate_yhi", "plate_T")]


class Numerics(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("dt", "Np", "r_p", "Kn_c", "pne_fixed")] + \
               [(n, C.c_int) for n in ("pne_mode", "n_avg", "avg_start", "precision",
                                       "weight_mode", "conserve_mode", "max_ppc", "jmom_mode",
                                       "spawn_projection", "window")] + \
               [("seed", C.c_uint64), ("avg_init", C.c_int), ("scheme", C.c_int),
                ("es_mode", C.c_int), ("gll_u", C.c_int), ("select_mode", C.c_int),
                ("es_sampler", C.c_int)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class MomentsView(C.Structure):
    _fields_ = [("ncell", C.c_int), ("nfield", C.c_int), ("data", C.c_void_p)]


class Stats(C.Structure):
    _fields_ = [("live", C.c_longlong), ("step", C.c_int), ("error", C.c_int),
                ("diag", C.c_int), ("added", C.c_longlong * 3)] + \
               [(n, C.c_longlong) for n in ("selected", "reassigned", "deleted", "entered",
                                            "left", "clamped", "es_fallback", "cells_invalid",
                                            "mass_fail", "energy_fail", "whole_cell")]


class Device(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", C.c_void_p),
                ("stream", C.c_void_p), ("device", C.c_int), ("budget", C.c_size_t)]


_lib = None


def lib():
    """Loads libusp.so (built by paper_1808_03801_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1808_03801_amd.build` (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        vp, ip, dp = C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_double)
        u32p = C.POINTER(C.c_uint32)
        sig = {
            "usp_create": (C.c_int, [C.POINTER(Device), C.POINTER(vp)]),
            "usp_destroy": (None, [vp]),
            "usp_last_error": (C.c_char_p, [vp]),
            "usp_footprint": (C.c_int, [C.POINTER(ProblemC), C.POINTER(Numerics),
                                        C.POINTER(C.c_size_t)]),
            "usp_instance_init": (C.c_int, [vp, C.POINTER(Gas), C.POINTER(ProblemC),
                                            C.POINTER(Numerics), dp, dp, dp, ip]),
            "usp_instance_free": (C.c_int, [vp, C.c_int]),
            "usp_step": (C.c_int, [vp, ip, C.c_int, C.c_int]),
            "usp_step_noalloc": (C.c_int, [vp, ip, C.c_int, C.c_int]),
            "usp_sync": (C.c_int, [vp]),
            "usp_instance_status": (C.c_int, [vp, C.c_int]),
            "usp_num_cells": (C.c_int, [vp, C.c_int, ip]),
            "usp_num_particles": (C.c_int, [vp, C.c_int, C.POINTER(C.c_longlong)]),
            "usp_get_state": (C.c_int, [vp, C.c_int, ip, dp, dp, ip, ip]),
            "usp_set_state": (C.c_int, [vp, C.c_int, ip, dp, dp, C.c_int, C.c_int]),
            "usp_get_fields": (C.c_int, [vp, C.c_int, C.c_int, dp]),
            "usp_set_diag": (C.c_int, [vp, C.c_int, C.c_int]),
            "usp_get_diag": (C.c_int, [vp, C.c_int, dp]),
            "usp_set_block": (C.c_int, [vp, C.c_int]),
            "usp_philox": (C.c_int, [vp, u32p, C.c_uint32, C.c_uint32, C.c_int, u32p]),
            "usp_set_timing": (C.c_int, [vp, C.c_int]),
            "usp_set_graph": (C.c_int, [vp, C.c_int]),
            "usp_set_shape": (C.c_int, [vp, C.c_int, C.c_int]),
            "usp_get_shape": (C.c_int, [vp, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                        C.POINTER(C.c_int)]),
            "usp_get_timing": (C.c_int, [vp, C.POINTER(C.c_double), C.POINTER(C.c_longlong)]),
            "usp_moments": (C.c_int, [vp, C.c_int, C.c_int, C.POINTER(MomentsView)]),
            "usp_get_sort": (C.c_int, [vp, C.c_int, C.POINTER(C.c_int32),
                                       C.POINTER(C.c_int32)]),
            "usp_stats": (C.c_int, [vp, C.c_int, C.POINTER(Stats)]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    """names the C header declares (for the load check)"""
    return ["usp_create", "usp_destroy", "usp_last_error", "usp_footprint", "usp_instance_init",
            "usp_instance_free", "usp_step", "usp_sync", "usp_instance_status", "usp_num_cells",
            "usp_num_particles", "usp_get_state", "usp_set_state", "usp_get_fields",
            "usp_set_diag", "usp_get_diag", "usp_set_block", "usp_philox", "usp_set_timing",
            "usp_get_timing", "usp_set_graph", "usp_set_shape", "usp_get_shape", "usp_moments",
            "usp_get_sort", "usp_stats", "usp_step_noalloc"]


_hiplib = None


def _hip():
    """the HIP runtime (already loaded by torch), for device-to-device copies
    of borrowed library buffers"""
    global _hiplib
    if _hiplib is None:
        _hiplib = C.CDLL("libamdhip64.so")
        _hiplib.hipMemcpyAsync.restype = C.c_int
        _hiplib.hipMemcpyAsync.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int,
                                           C.c_void_p]
    return _hiplib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


def to_c(pb):
    """(Gas, ProblemC, Numerics) of a problems.Problem"""
    g = pb.gas
    gas = Gas(g.m, g.kB, g.mu_ref, g.T_ref, g.omega, g.Pr)
    p = ProblemC()
    p.dim, p.nx, p.ny = pb.dim, pb.nx, pb.ny
    for n in ("x0", "x1", "y0", "y1", "dx", "dy", "inv_dx", "inv_dy", "vcell"):
        setattr(p, n, getattr(pb, n))
    for i, f in enumerate(pb.faces):
        p.face[i].kind = f.kind
        p.face[i].T = f.T
        for k in range(3):
            p.face[i].u[k] = f.u[k]
        p.face[i].n, p.face[i].split, p.face[i].n_b, p.face[i].T_b = f.n, f.split, f.n_b, f.T_b
    for k in range(3):
        p.accel[k] = pb.accel[k]
    p.plate, p.plate_x, p.plate_ylo, p.plate_yhi, p.plate_T = (pb.plate, pb.plate_x, pb.plate_ylo,
                                                              pb.plate_yhi, pb.plate_T)
    nm = Numerics()
    for n in ("dt", "Np", "r_p", "Kn_c", "pne_fixed"):
        setattr(nm, n, getattr(pb, n))
    for n in ("pne_mode", "n_avg", "avg_start", "precision", "weight_mode", "conserve_mode",
              "max_ppc", "jmom_mode", "spawn_projection"):
        setattr(nm, n, int(getattr(pb, n)))
    nm.window = int(pb.meta.get("window", 0))
    nm.seed = int(pb.seed)
    nm.avg_init = int(pb.avg_init)
    nm.scheme = int(pb.scheme)
    nm.es_mode = int(pb.es_mode)
    nm.gll_u = int(pb.gll_u)
    nm.select_mode = int(pb.select_mode)
    nm.es_sampler = int(pb.es_sampler)
    return gas, p, nm


def footprint(pb) -> int:
    _, p, nm = to_c(pb)
    out = C.c_size_t()
    _check(None, lib().usp_footprint(C.byref(p), C.byref(nm), C.byref(out)))
    return out.value


def _check(ctx, status):
    if status != 0:
        msg = lib().usp_last_error(ctx).decode() if ctx else ""
        raise UspError(status, msg)


class State:
    """Host copy of a solver state (same layout as the C-ABI)."""

    def __init__(self, counts, parts, cells, step, n_samples):
        self.counts = np.ascontiguousarray(counts, dtype=np.int32)
        self.parts = np.ascontiguousarray(parts, dtype=np.float64).reshape(-1, 6)
        self.cells = None if cells is None else np.ascontiguousarray(cells, dtype=np.float64)
        self.step = int(step)
        self.n_samples = int(n_samples)

    @property
    def offsets(self):
        return np.concatenate([[0], np.cumsum(self.counts)])


class Context:
    """One device + stream.  By default device memory comes from PyTorch's
    caching allocator and work goes on PyTorch's current stream."""

    def __init__(self, device: int = 0, use_torch: bool = True, budget: int = 0, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libusp needs a ROCm GPU; none is visible")
        self.torch = torch
        self.device = device
        self._live = {}
        dev = Device()
        dev.device = device
        dev.budget = budget
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        dev.stream = C.c_void_p(stream.cuda_stream)
        if use_torch:
            def _alloc(nbytes, user):
                ptr = torch.cuda.caching_allocator_alloc(int(nbytes), device, stream)
                self._live[ptr] = nbytes
                return ptr

            def _free(ptr, user):
                if ptr in self._live:
                    del self._live[ptr]
                    torch.cuda.caching_allocator_delete(ptr)

            self._alloc_cb = ALLOC_FN(_alloc)
            self._free_cb = FREE_FN(_free)
            dev.alloc = self._alloc_cb
            dev.free = self._free_cb
        h = C.c_void_p()
        _check(None, lib().usp_create(C.byref(dev), C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().usp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add(self, pb) -> "Instance":
        gas, p, nm = to_c(pb)
        n = np.ascontiguousarray(pb.init_n, dtype=np.float64)
        u = np.ascontiguousarray(pb.init_u, dtype=np.float64).reshape(-1)
        T = np.ascontiguousarray(pb.init_T, dtype=np.float64)
        iid = C.c_int()
        _check(self.h, lib().usp_instance_init(self.h, C.byref(gas), C.byref(p), C.byref(nm),
                                              _dp(n), _dp(u), _dp(T), C.byref(iid)))
        return Instance(self, iid.value, pb)

    def step(self, instances, nsteps: int = 1):
        ids = np.array([i.id for i in instances], dtype=np.int32)
        _check(self.h, lib().usp_step(self.h, _ip(ids), len(ids), int(nsteps)))

    def step_noalloc(self, instances, nsteps: int = 1):
        """usp_step without device allocation (static scratch; see the header)"""
        ids = np.array([i.id for i in instances], dtype=np.int32)
        _check(self.h, lib().usp_step_noalloc(self.h, _ip(ids), len(ids), int(nsteps)))

    def sync(self):
        _check(self.h, lib().usp_sync(self.h))

    def set_block(self, threads: int):
        _check(self.h, lib().usp_set_block(self.h, int(threads)))

    def set_timing(self, on: bool):
        _check(self.h, lib().usp_set_timing(self.h, int(on)))

    def set_graph(self, on: bool):
        """capture each distinct step call into a HIP graph and replay it"""
        _check(self.h, lib().usp_set_graph(self.h, int(on)))

    def timing(self):
        """(summed cell-kernel time in ms, number of cell passes)"""
        ms, n = C.c_double(), C.c_longlong()
        _check(self.h, lib().usp_get_timing(self.h, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def philox(self, ctr, key):
        ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
        out = np.zeros_like(ctr)
        u32p = C.POINTER(C.c_uint32)
        _check(self.h, lib().usp_philox(self.h, ctr.ctypes.data_as(u32p), int(key[0]),
                                        int(key[1]), ctr.shape[0], out.ctypes.data_as(u32p)))
        return out


class Instance:
    def __init__(self, ctx: Context, iid: int, pb):
        self.ctx = ctx
        self.id = iid
        self.pb = pb
        self.ncell = pb.nx * pb.ny

    def step(self, nsteps: int = 1):
        self.ctx.step([self], nsteps)

    def status(self) -> int:
        return lib().usp_instance_status(self.ctx.h, self.id)

    def num_particles(self) -> int:
        n = C.c_longlong()
        _check(self.ctx.h, lib().usp_num_particles(self.ctx.h, self.id, C.byref(n)))
        return n.value

    def get_state(self, with_parts=True) -> State:
        counts = np.zeros(self.ncell, np.int32)
        L = lib()
        st, ns = C.c_int(), C.c_int()
        _check(self.ctx.h, L.usp_get_state(self.ctx.h, self.id, _ip(counts), None, None,
                                           C.byref(st), C.byref(ns)))
        N = int(counts.sum())
        parts = np.zeros((max(N, 1), 6))
        cells = np.zeros((self.ncell, NCS))
        _check(self.ctx.h, L.usp_get_state(self.ctx.h, self.id, _ip(counts),
                                           _dp(parts) if with_parts else None, _dp(cells),
                                           C.byref(st), C.byref(ns)))
        return State(counts, parts[:N], cells, st.value, ns.value)

    def set_state(self, s):
        parts = np.ascontiguousarray(s.parts, dtype=np.float64).reshape(-1, 6)
        if parts.shape[0] == 0:
            parts = np.zeros((1, 6))
        counts = np.ascontiguousarray(s.counts, dtype=np.int32)
        cells = None if s.cells is None else np.ascontiguousarray(s.cells, dtype=np.float64)
        _check(self.ctx.h, lib().usp_set_state(self.ctx.h, self.id, _ip(counts), _dp(parts),
                                               None if cells is None else _dp(cells),
                                               int(s.step), int(s.n_samples)))

    def fields(self, which: int = 0):
        out = np.zeros((self.ncell, NF))
        _check(self.ctx.h, lib().usp_get_fields(self.ctx.h, self.id, which, _dp(out)))
        return out

    def moments_view(self, which: int = 0):
        """usp_moments: (ncell, nfield, device address of the field-major
        [nfield][ncell] FP64 record), borrowed until the next step"""
        v = MomentsView()
        _check(self.ctx.h, lib().usp_moments(self.ctx.h, self.id, which, C.byref(v)))
        return v.ncell, v.nfield, v.data

    def moments_device(self, which: int = 0):
        """the usp_moments record as a torch tensor [nfield][ncell] (a copy
        on the device, made on the library's stream)"""
        import torch
        ncell, nfield, ptr = self.moments_view(which)
        out = torch.empty((nfield, ncell), dtype=torch.float64, device=f"cuda:{self.ctx.device}")
        rc = _hip().hipMemcpyAsync(C.c_void_p(out.data_ptr()), C.c_void_p(ptr),
                                   C.c_size_t(nfield * ncell * 8), 3,
                                   C.c_void_p(self.ctx.stream.cuda_stream))
        if rc != 0:
            raise UspError(-5, f"hipMemcpyAsync failed ({rc})")
        return out

    def set_diag(self, on=True):
        _check(self.ctx.h, lib().usp_set_diag(self.ctx.h, self.id, int(on)))

    def diag(self):
        out = np.zeros((self.ncell, NDIAG))
        _check(self.ctx.h, lib().usp_get_diag(self.ctx.h, self.id, _dp(out)))
        return out

    def get_sort(self):
        """usp_get_sort: (counts per cell after the last step-3 sort, place of
        every sorted particle in the sequence before it)"""
        off = np.zeros(self.ncell + 1, np.int32)
        i32p = C.POINTER(C.c_int32)
        _check(self.ctx.h, lib().usp_get_sort(self.ctx.h, self.id, off.ctypes.data_as(i32p),
                                              None))
        perm = np.zeros(max(int(off[-1]), 1), np.int32)
        _check(self.ctx.h, lib().usp_get_sort(self.ctx.h, self.id, off.ctypes.data_as(i32p),
                                              perm.ctypes.data_as(i32p)))
        return np.diff(off).astype(np.int32), perm[:int(off[-1])].astype(np.int64)

    def stats(self) -> dict:
        """usp_stats as a dict"""
        st = Stats()
        _check(self.ctx.h, lib().usp_stats(self.ctx.h, self.id, C.byref(st)))
        d = {n: getattr(st, n) for n, _ in Stats._fields_ if n != "added"}
        d["added"] = list(st.added)
        return d

    def set_shape(self, first: int):
        """first launch shape of this instance (-1: default); results unchanged"""
        _check(self.ctx.h, lib().usp_set_shape(self.ctx.h, self.id, int(first)))

    def shape(self):
        """(first shape, last shape, number of shapes)"""
        a, b, n = C.c_int(), C.c_int(), C.c_int()
        _check(self.ctx.h, lib().usp_get_shape(self.ctx.h, self.id, C.byref(a), C.byref(b),
                                               C.byref(n)))
        return a.value, b.value, n.value

    def free(self):
        _check(self.ctx.h, lib().usp_instance_free(self.ctx.h, self.id))
