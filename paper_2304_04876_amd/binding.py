"""ctypes binding of libgdsw.so (C ABI in include/gdsw.h).

Argument marshalling only: every step of the preconditioner runs in the
library (host analysis in C++, numerical setup, applies and solves in HIP
kernels).  Functions keep the C names; device vectors may be passed as torch
tensors (FP64, on the GPU) or raw device addresses, streams as
``torch.cuda.Stream`` objects, raw ``hipStream_t`` addresses or None (the
current torch stream).  If the library has not been built, ``lib()`` raises;
there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgdsw.so")
_LIB = None

GDSW_OK = 0
STATUS_NAMES = {0: "OK", 1: "INVALID_ARG", 2: "SINGULAR", 3: "BREAKDOWN", 4: "NOT_CONVERGED",
                5: "BUDGET", 6: "HIP", 7: "STATE", 8: "INTERNAL"}
COARSE_NONE, COARSE_GDSW, COARSE_RGDSW = 0, 1, 2
LOCAL_EXACT, LOCAL_ILU0 = 0, 1
FP64, FP32, BF16, FP16 = 0, 1, 2, 3
KRYLOV_CG, KRYLOV_GMRES, KRYLOV_GMRES_SR = 0, 1, 2
FLAG_GRAPHS = 1
MAP_OV_PTR, MAP_OV_IDX, MAP_IS_GAMMA, MAP_COMP_OF_NODE, MAP_COMP_RANK = 0, 1, 2, 3, 4
MAP_PHI_ROWPTR, MAP_PHI_COL, MAP_PHI_VAL, MAP_A0 = 5, 6, 7, 8
MAP_LOCAL_ROWPTR, MAP_LOCAL_COL = 9, 10
(MAP_ND_PERM, MAP_ND_SN_PTR, MAP_ND_SN, MAP_ND_VOFF, MAP_ND_ST_PTR, MAP_ND_ST_ROW, MAP_ND_RC_PTR, MAP_ND_RC,
 MAP_ND_LV_BASE, MAP_ND_LV_PTR, MAP_ND_LV_ROWS, MAP_ND_UP_PTR, MAP_ND_UP, MAP_ND_REL, MAP_ND_ASM,
 MAP_ND_RC_W, MAP_ND_ST_SN, MAP_ND_LV_INFO, MAP_ND_CH_BASE, MAP_ND_CH_ROW) = range(11, 31)
_MAP_DTYPE = {0: np.int64, 1: np.int64, 2: np.int8, 3: np.int32, 4: np.int32,
              5: np.int64, 6: np.int32, 7: np.float64, 8: np.float64, 9: np.int64, 10: np.int32,
              11: np.int32, 12: np.int64, 13: np.int32, 14: np.int64, 15: np.int64, 16: np.int32, 17: np.int64,
              18: np.int32, 19: np.int64, 20: np.int32, 21: np.int32, 22: np.int64, 23: np.int64, 24: np.int32,
              25: np.int64, 26: np.int32, 27: np.int32, 28: np.int32, 29: np.int64, 30: np.int32}
ORDER_NATURAL, ORDER_ND, ORDER_AUTO = 0, 1, 2

EXPORTED = ("gdsw_default_options", "gdsw_analyze", "gdsw_analyze_sharing", "gdsw_factor", "gdsw_refactor",
            "gdsw_setup", "gdsw_apply", "gdsw_apply_static", "gdsw_apply_part", "gdsw_spmv", "gdsw_solve", "gdsw_get_info",
            "gdsw_map_size", "gdsw_copy_map", "gdsw_destroy", "gdsw_status_string", "gdsw_last_error",
            "gdsw_analyze_batch", "gdsw_solve_batch", "gdsw_slots_begin", "gdsw_slot_start",
            "gdsw_slots_step", "gdsw_slot_finish", "gdsw_problem_offsets", "gdsw_autotune", "gdsw_set_launch",
            "gdsw_set_size_classes", "gdsw_profile_local", "gdsw_profile_read")


class Options(ctypes.Structure):
    _fields_ = [("overlap", ctypes.c_int32), ("coarse", ctypes.c_int32), ("local", ctypes.c_int32),
                ("jacobi_sweeps", ctypes.c_int32), ("local_prec", ctypes.c_int32),
                ("basis_prec", ctypes.c_int32), ("hbm_budget_bytes", ctypes.c_int64),
                ("flags", ctypes.c_uint64), ("ilu_level", ctypes.c_int32),
                ("ilu_factor_sweeps", ctypes.c_int32), ("slots", ctypes.c_int32),
                ("exact_order", ctypes.c_int32)]


class CSR(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("rowptr", ctypes.c_void_p), ("col", ctypes.c_void_p),
                ("val", ctypes.c_void_p)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("rel_res_recursive", ctypes.c_double), ("rel_res_true", ctypes.c_double),
                ("seconds", ctypes.c_double)]


class Info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("n_nodes", ctypes.c_int64), ("dpn", ctypes.c_int32),
                ("n_parts", ctypes.c_int32), ("sum_overlap_dofs", ctypes.c_int64),
                ("n_gamma_nodes", ctypes.c_int64), ("n_components", ctypes.c_int32),
                ("n0", ctypes.c_int32), ("local_factor_entries", ctypes.c_int64),
                ("phi_entries", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("max_local_rows", ctypes.c_int32), ("max_bandwidth", ctypes.c_int32),
                ("t_analyze", ctypes.c_double), ("t_factor", ctypes.c_double),
                ("n_problems", ctypes.c_int32), ("local_variant", ctypes.c_int32),
                ("gemv_variant", ctypes.c_int32), ("apply_streams", ctypes.c_int32),
                ("prolong_variant", ctypes.c_int32), ("t_refactor", ctypes.c_double),
                ("slots", ctypes.c_int32), ("slot_bytes", ctypes.c_int64), ("exact_order", ctypes.c_int32),
                ("nd_subdomains", ctypes.c_int32), ("local_classes", ctypes.c_int32),
                ("local_solve_bytes", ctypes.c_int64)]


def lib():
    """Loads libgdsw.so; raises RuntimeError if it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2304_04876_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "gdsw_default_options": (None, [ctypes.POINTER(Options)]),
        "gdsw_analyze": (ctypes.c_int, [ctypes.POINTER(CSR), vp, i32, i32, vp, i32, ctypes.POINTER(Options),
                                        ctypes.POINTER(vp)]),
        "gdsw_analyze_sharing": (ctypes.c_int, [ctypes.POINTER(CSR), vp, i32, i32, vp, i32, vp, vp,
                                                ctypes.POINTER(Options), ctypes.POINTER(vp)]),
        "gdsw_factor": (ctypes.c_int, [vp, vp]),
        "gdsw_refactor": (ctypes.c_int, [vp, vp, vp]),
        "gdsw_setup": (ctypes.c_int, [ctypes.POINTER(CSR), vp, i32, i32, vp, i32, ctypes.POINTER(Options), vp,
                                      ctypes.POINTER(vp)]),
        "gdsw_apply": (ctypes.c_int, [vp, vp, vp, vp]),
        "gdsw_apply_part": (ctypes.c_int, [vp, vp, vp, i32, vp]),
        "gdsw_apply_static": (ctypes.c_int, [vp, vp, vp, vp]),
        "gdsw_spmv": (ctypes.c_int, [vp, vp, vp, vp]),
        "gdsw_solve": (ctypes.c_int, [vp, vp, vp, i32, i32, dbl, i32, i32, ctypes.POINTER(SolveInfo), vp]),
        "gdsw_get_info": (ctypes.c_int, [vp, ctypes.POINTER(Info)]),
        "gdsw_map_size": (ctypes.c_int, [vp, i32, ctypes.POINTER(i64)]),
        "gdsw_copy_map": (ctypes.c_int, [vp, i32, vp]),
        "gdsw_destroy": (ctypes.c_int, [vp]),
        "gdsw_status_string": (ctypes.c_char_p, [ctypes.c_int]),
        "gdsw_analyze_batch": (ctypes.c_int, [i32, ctypes.POINTER(CSR), ctypes.POINTER(vp), vp, i32,
                                              ctypes.POINTER(vp), i32, ctypes.POINTER(Options),
                                              ctypes.POINTER(vp)]),
        "gdsw_solve_batch": (ctypes.c_int, [vp, vp, vp, dbl, i32, ctypes.POINTER(SolveInfo), vp]),
        "gdsw_slots_begin": (ctypes.c_int, [vp, vp, vp, dbl, i32, vp]),
        "gdsw_slot_start": (ctypes.c_int, [vp, i32, vp]),
        "gdsw_slots_step": (ctypes.c_int, [vp, i32, vp, vp]),
        "gdsw_slot_finish": (ctypes.c_int, [vp, i32, ctypes.POINTER(SolveInfo), vp]),
        "gdsw_problem_offsets": (ctypes.c_int, [vp, vp]),
        "gdsw_autotune": (ctypes.c_int, [vp, i32, vp, vp]),
        "gdsw_set_launch": (ctypes.c_int, [vp, i32, i32, i32, i32, vp]),
        "gdsw_set_size_classes": (ctypes.c_int, [vp, i32]),
        "gdsw_profile_local": (ctypes.c_int, [vp, i32]),
        "gdsw_profile_read": (ctypes.c_int, [vp, vp, i32, vp]),
        "gdsw_last_error": (ctypes.c_char_p, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _LIB = L
    return L


class GdswError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _ptr(x):
    """Device address of a torch tensor, or an int address, or None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(s):
    if s is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(s, int):
        return s
    return s.cuda_stream


def gdsw_default_options(**kw) -> Options:
    o = Options()
    lib().gdsw_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def _csr_arrays(A):
    A = A.tocsr()
    A.sort_indices()
    rowptr = np.ascontiguousarray(A.indptr, dtype=np.int64)
    col = np.ascontiguousarray(A.indices, dtype=np.int32)
    val = np.ascontiguousarray(A.data, dtype=np.float64)
    return rowptr, col, val


def gdsw_analyze(A, part, n_parts, dpn=1, Z=None, options: Options | None = None, sharing=None):
    """Symbolic phase on the host; returns a handle (int).  sharing: None
    (the interface from the node graph) or (share_ptr, share_sub), the sets
    of subdomains sharing each node (gdsw_analyze_sharing)."""
    rowptr, col, val = _csr_arrays(A)
    csr = CSR(A.shape[0], rowptr.ctypes.data, col.ctypes.data, val.ctypes.data)
    part = np.ascontiguousarray(part, dtype=np.int32)
    if Z is not None:
        Zc = np.asfortranarray(np.asarray(Z, dtype=np.float64).reshape(A.shape[0], -1))
        zp, nz = Zc.ctypes.data, Zc.shape[1]
    else:
        Zc, zp, nz = None, None, 0
    opt = options if options is not None else gdsw_default_options()
    h = ctypes.c_void_p()
    if sharing is None:
        st = lib().gdsw_analyze(ctypes.byref(csr), part.ctypes.data, int(n_parts), int(dpn), zp, nz,
                                ctypes.byref(opt), ctypes.byref(h))
    else:
        sp_ = np.ascontiguousarray(sharing[0], dtype=np.int64)
        ss_ = np.ascontiguousarray(sharing[1], dtype=np.int32)
        st = lib().gdsw_analyze_sharing(ctypes.byref(csr), part.ctypes.data, int(n_parts), int(dpn), zp, nz,
                                        sp_.ctypes.data, ss_.ctypes.data if ss_.size else sp_.ctypes.data,
                                        ctypes.byref(opt), ctypes.byref(h))
    if st != GDSW_OK:
        msg = gdsw_last_error(h.value)
        gdsw_destroy(h.value)
        raise GdswError(st, msg)
    return h.value


def _check(h, st):
    if st != GDSW_OK:
        raise GdswError(st, gdsw_last_error(h))


def gdsw_factor(h, stream=None):
    _check(h, lib().gdsw_factor(h, _stream(stream)))


def gdsw_refactor(h, val, stream=None):
    v = np.ascontiguousarray(val, dtype=np.float64)
    _check(h, lib().gdsw_refactor(h, v.ctypes.data, _stream(stream)))


def gdsw_setup(A, part, n_parts, dpn=1, Z=None, options=None, stream=None):
    h = gdsw_analyze(A, part, n_parts, dpn, Z, options)
    try:
        gdsw_factor(h, stream)
    except Exception:
        gdsw_destroy(h)
        raise
    return h


def gdsw_apply(h, r, z, stream=None):
    _check(h, lib().gdsw_apply(h, _ptr(r), _ptr(z), _stream(stream)))


def gdsw_apply_static(h, r, z, stream=None):
    _check(h, lib().gdsw_apply_static(h, _ptr(r), _ptr(z), _stream(stream)))


def gdsw_apply_part(h, r, z, which, stream=None):
    _check(h, lib().gdsw_apply_part(h, _ptr(r), _ptr(z), int(which), _stream(stream)))


def gdsw_spmv(h, x, y, stream=None):
    _check(h, lib().gdsw_spmv(h, _ptr(x), _ptr(y), _stream(stream)))


def gdsw_solve(h, b, x, krylov=KRYLOV_CG, restart=30, rtol=1e-8, maxit=1000, fixed_iters=0,
               stream=None, raise_on_error=True):
    info = SolveInfo()
    st = lib().gdsw_solve(h, _ptr(b), _ptr(x), int(krylov), int(restart), float(rtol), int(maxit),
                          int(fixed_iters), ctypes.byref(info), _stream(stream))
    out = {"status": st, "iterations": info.iterations, "converged": bool(info.converged),
           "rel_res_recursive": info.rel_res_recursive, "rel_res_true": info.rel_res_true,
           "seconds": info.seconds}
    if raise_on_error and st != GDSW_OK:
        raise GdswError(st, gdsw_last_error(h))
    return out


def gdsw_analyze_batch(problems, dpn=1, Z=None, options: Options | None = None):
    """Symbolic phase of a batch of independent problems; ``problems`` is a
    list of (A, part, n_parts).  ``Z``: None or a list of null-space blocks."""
    count = len(problems)
    keep = []
    csrs = (CSR * count)()
    parts = (ctypes.c_void_p * count)()
    nparts = np.zeros(count, dtype=np.int32)
    for k, (A, part, npk) in enumerate(problems):
        rowptr, col, val = _csr_arrays(A)
        p = np.ascontiguousarray(part, dtype=np.int32)
        keep += [rowptr, col, val, p]
        csrs[k] = CSR(A.shape[0], rowptr.ctypes.data, col.ctypes.data, val.ctypes.data)
        parts[k] = p.ctypes.data
        nparts[k] = npk
    zp = None
    nz = 0
    if Z is not None:
        zarr = (ctypes.c_void_p * count)()
        for k, zk in enumerate(Z):
            zk = np.asfortranarray(np.asarray(zk, dtype=np.float64))
            keep.append(zk)
            zarr[k] = zk.ctypes.data
            nz = zk.shape[1]
        zp = zarr
    opt = options if options is not None else gdsw_default_options()
    h = ctypes.c_void_p()
    st = lib().gdsw_analyze_batch(count, csrs, parts, nparts.ctypes.data, int(dpn), zp, nz,
                                  ctypes.byref(opt), ctypes.byref(h))
    if st != GDSW_OK:
        msg = gdsw_last_error(h.value)
        gdsw_destroy(h.value)
        raise GdswError(st, msg)
    return h.value


def _info_dict(info, st=None):
    d = {"iterations": info.iterations, "converged": bool(info.converged),
         "rel_res_recursive": info.rel_res_recursive, "rel_res_true": info.rel_res_true,
         "seconds": info.seconds}
    if st is not None:
        d["status"] = st
    return d


def _krylov_problems(h):
    """(slot, problem) pairs of a handle: slots * n_problems."""
    inf = gdsw_get_info(h)
    return inf["n_problems"] * max(1, inf["slots"])


def gdsw_solve_batch(h, b, x, rtol=1e-8, maxit=1000, stream=None, raise_on_error=True):
    count = _krylov_problems(h)
    infos = (SolveInfo * count)()
    st = lib().gdsw_solve_batch(h, _ptr(b), _ptr(x), float(rtol), int(maxit), infos, _stream(stream))
    if raise_on_error and st != GDSW_OK:
        raise GdswError(st, gdsw_last_error(h))
    return [_info_dict(i) for i in infos]


def gdsw_slots_begin(h, b, x, rtol=1e-8, maxit=1000, stream=None):
    _check(h, lib().gdsw_slots_begin(h, _ptr(b), _ptr(x), float(rtol), int(maxit), _stream(stream)))


def gdsw_slot_start(h, slot, stream=None):
    _check(h, lib().gdsw_slot_start(h, int(slot), _stream(stream)))


def gdsw_slots_step(h, iters, stream=None) -> np.ndarray:
    count = _krylov_problems(h)
    state = np.zeros(count, dtype=np.int32)
    _check(h, lib().gdsw_slots_step(h, int(iters), state.ctypes.data, _stream(stream)))
    return state


def gdsw_slot_finish(h, slot, stream=None) -> dict:
    info = SolveInfo()
    st = lib().gdsw_slot_finish(h, int(slot), ctypes.byref(info), _stream(stream))
    if st not in (GDSW_OK, 3, 4):
        raise GdswError(st, gdsw_last_error(h))
    return _info_dict(info, st)


def gdsw_autotune(h, reps=10, stream=None) -> list:
    times = np.full(16, -1.0, dtype=np.float32)
    _check(h, lib().gdsw_autotune(h, int(reps), times.ctypes.data, _stream(stream)))
    return times.tolist()


def gdsw_set_size_classes(h, split):
    _check(h, lib().gdsw_set_size_classes(h, int(split)))


def gdsw_set_launch(h, local_variant=-1, gemv_variant=-1, apply_streams=-1, prolong_variant=-1, stream=None):
    _check(h, lib().gdsw_set_launch(h, int(local_variant), int(gemv_variant), int(apply_streams),
                                    int(prolong_variant), _stream(stream)))


PROFILE_MAX = 1024


def gdsw_profile_local(h, enable=True):
    _check(h, lib().gdsw_profile_local(h, 1 if enable else 0))


def gdsw_profile_read(h) -> np.ndarray:
    """Milliseconds of each recorded local-solve launch (waits for them)."""
    ms = np.zeros(PROFILE_MAX, dtype=np.float32)
    count = ctypes.c_int32(0)
    _check(h, lib().gdsw_profile_read(h, ms.ctypes.data, PROFILE_MAX, ctypes.byref(count)))
    return ms[:min(count.value, PROFILE_MAX)].astype(np.float64)


def gdsw_problem_offsets(h) -> np.ndarray:
    count = _krylov_problems(h)
    out = np.zeros(count + 1, dtype=np.int64)
    _check(h, lib().gdsw_problem_offsets(h, out.ctypes.data))
    return out


def gdsw_get_info(h) -> dict:
    info = Info()
    _check(h, lib().gdsw_get_info(h, ctypes.byref(info)))
    return {name: getattr(info, name) for name, _ in Info._fields_}


def gdsw_map_size(h, which) -> int:
    c = ctypes.c_int64()
    _check(h, lib().gdsw_map_size(h, int(which), ctypes.byref(c)))
    return c.value


def gdsw_copy_map(h, which) -> np.ndarray:
    out = np.empty(max(gdsw_map_size(h, which), 1), dtype=_MAP_DTYPE[which])
    _check(h, lib().gdsw_copy_map(h, int(which), out.ctypes.data))
    return out[:gdsw_map_size(h, which)]


def gdsw_destroy(h):
    if h:
        lib().gdsw_destroy(h)


def gdsw_status_string(st) -> str:
    return lib().gdsw_status_string(int(st)).decode()


def gdsw_last_error(h) -> str:
    m = lib().gdsw_last_error(h)
    return m.decode() if m else ""


class Gdsw:
    """Owning wrapper of a handle (destroyed with the object)."""

    def __init__(self, A, part, n_parts, dpn=1, Z=None, factor=True, stream=None, sharing=None, **options):
        self.h = gdsw_analyze(A, part, n_parts, dpn, Z, gdsw_default_options(**options), sharing=sharing)
        self.n = A.shape[0]
        if factor:
            try:
                gdsw_factor(self.h, stream)
            except Exception:
                self.close()
                raise

    def apply(self, r, z, stream=None):
        gdsw_apply(self.h, r, z, stream)

    def apply_part(self, r, z, which, stream=None):
        gdsw_apply_part(self.h, r, z, which, stream)

    def spmv(self, x, y, stream=None):
        gdsw_spmv(self.h, x, y, stream)

    def solve(self, b, x, **kw):
        return gdsw_solve(self.h, b, x, **kw)

    def info(self):
        return gdsw_get_info(self.h)

    def map(self, which):
        return gdsw_copy_map(self.h, which)

    def close(self):
        if getattr(self, "h", None):
            gdsw_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
