"""Thin ctypes binding of liblspr.so (the C ABI declared in include/lspr.h).

Argument marshalling only: every step of the method runs inside the HIP library.  PyTorch is
used for device memory and streams (tensor.data_ptr(), torch.cuda.current_stream()).  The
library must have been built (paper_1812_10722_amd/build.py); importing this module without it
raises ImportError -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
# torch first: its HIP runtime is then the one this library binds to, whatever the caller
# imports next (two runtimes in one process do not see the same device)
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblspr.so")

LSPR_OK, LSPR_E_INVALID, LSPR_E_MESH, LSPR_E_NOMEM, LSPR_E_DEVICE, LSPR_E_NOCONV, LSPR_E_BUSY = range(7)
LSPR_DENSE, LSPR_TREECODE = 0, 1
LSPR_FP64, LSPR_FP32, LSPR_FP32_REFINE64, LSPR_FP32_LEAD64 = 0, 1, 2, 3
_PRECISION = {"fp64": LSPR_FP64, "fp32": LSPR_FP32, "fp32_refine64": LSPR_FP32_REFINE64,
              "fp32_lead64": LSPR_FP32_LEAD64}


class lspr_c64(C.Structure):
    _fields_ = [("re", C.c_double), ("im", C.c_double)]


class lspr_surface(C.Structure):
    _fields_ = [("n_vert", C.c_int32), ("vert", C.c_void_p), ("n_tri", C.c_int32),
                ("tri", C.c_void_p)]


class lspr_op_params(C.Structure):
    _fields_ = [("k_far", C.c_int32), ("k_fine", C.c_int32), ("n_k", C.c_int32),
                ("threshold", C.c_double), ("method", C.c_int32), ("p", C.c_int32),
                ("theta", C.c_double), ("ncrit", C.c_int32), ("precision", C.c_int32),
                ("m2p_min_panels", C.c_int32), ("flags", C.c_int32)]


class lspr_gmres_params(C.Structure):
    _fields_ = [("tol", C.c_double), ("restart", C.c_int32), ("max_iter", C.c_int32),
                ("precond", C.c_int32), ("inner_tol", C.c_double)]


class lspr_geometry_stats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in (
        "n_panels", "n_surfaces", "n_nodes", "n_boxes", "n_leaves", "n_target_chunks", "n_m2p",
        "n_p2p_ranges", "p2p_pairs", "m2p_pairs", "n_near", "device_bytes")] + \
        [(n, C.c_int32) for n in ("n_terms", "ncrit", "target_chunk", "max_depth")] + \
        [(n, C.c_int64) for n in ("n_tiles", "tile_steps", "max_chunk_steps")]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_1812_10722_amd/build.py")
    lib = C.CDLL(LIB_PATH)
    vp, i32, dbl = C.c_void_p, C.c_int32, C.c_double
    P = C.POINTER
    sig = {
        "lspr_mesh_validate": (C.c_int, [P(lspr_surface), i32]),
        "lspr_geometry_create": (C.c_int, [P(lspr_surface), i32, P(lspr_op_params), vp, P(vp)]),
        "lspr_geometry_destroy": (C.c_int, [vp]),
        "lspr_geometry_info": (C.c_int, [vp, P(lspr_geometry_stats)]),
        "lspr_geometry_set_charges": (C.c_int, [vp, i32, P(dbl), P(dbl), P(i32), vp]),
        "lspr_solve": (C.c_int, [vp, i32, P(dbl), P(lspr_c64), P(lspr_c64), P(dbl),
                                 P(lspr_gmres_params), vp, vp, vp, P(lspr_c64), P(lspr_c64),
                                 P(dbl), P(dbl), P(i32), P(dbl)]),
        "lspr_apply": (C.c_int, [vp, i32, P(lspr_c64), P(lspr_c64), vp, vp, vp]),
        "lspr_apply_noalloc": (C.c_int, [vp, i32, P(lspr_c64), P(lspr_c64), vp, vp, vp]),
        "lspr_rhs": (C.c_int, [vp, i32, P(lspr_c64), P(lspr_c64), P(dbl), vp, vp]),
        "lspr_triangle_rule": (C.c_int, [i32, P(dbl), P(dbl)]),
        "lspr_gauss_legendre": (C.c_int, [i32, P(dbl), P(dbl)]),
        "lspr_resonance_peak": (C.c_int, [i32, P(dbl), P(dbl), P(dbl), P(dbl)]),
        "lspr_status_string": (C.c_char_p, [C.c_int]),
        "lspr_last_error": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load()


class LsprError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        msg = _lib.lspr_last_error().decode()
        super().__init__(f"{where}: {_lib.lspr_status_string(code).decode()} ({code}): {msg}")


def _check(code, where, allow=()):
    if code != LSPR_OK and code not in allow:
        raise LsprError(code, where)
    return code


def _dptr(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def _c64_array(z):
    z = np.ascontiguousarray(np.asarray(z, dtype=np.complex128))
    return z, z.ctypes.data_as(C.POINTER(lspr_c64))


# ------------------------------------------------------------------ functions with the C names
def lspr_triangle_rule(n: int):
    bary = np.zeros((n, 3))
    w = np.zeros(n)
    _check(_lib.lspr_triangle_rule(n, _dptr(bary), _dptr(w)), "lspr_triangle_rule")
    return bary, w


def lspr_gauss_legendre(n: int):
    t = np.zeros(n)
    w = np.zeros(n)
    _check(_lib.lspr_gauss_legendre(n, _dptr(t), _dptr(w)), "lspr_gauss_legendre")
    return t, w


def lspr_resonance_peak(lambdas, cext):
    """(peak wavelength, peak C_ext) of a sampled spectrum (parabola through the maximum)."""
    lam = np.ascontiguousarray(lambdas, dtype=np.float64)
    c = np.ascontiguousarray(cext, dtype=np.float64)
    pl, pc = C.c_double(), C.c_double()
    _check(_lib.lspr_resonance_peak(len(lam), _dptr(lam), _dptr(c), C.byref(pl), C.byref(pc)),
           "lspr_resonance_peak")
    return pl.value, pc.value


def lspr_mesh_validate(surfaces):
    """surfaces: list of (verts [n,3] float64, tris [m,3] int32) host arrays."""
    keep = []
    arr = (lspr_surface * len(surfaces))()
    for k, (v, t) in enumerate(surfaces):
        v = np.ascontiguousarray(v, dtype=np.float64)
        t = np.ascontiguousarray(t, dtype=np.int32)
        keep += [v, t]
        arr[k] = lspr_surface(len(v), v.ctypes.data, len(t), t.ctypes.data)
    return _lib.lspr_mesh_validate(arr, len(surfaces))


def _stream_ptr(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


LSPR_NO_MATRIX_CORES = 1
LSPR_STREAM_NARROW = 4
LSPR_PAIR_OPERATORS = 8
LSPR_PAIR_NARROW = 16
LSPR_FOUR_WAVE = 32


def op_params(k_far=4, k_fine=19, n_k=9, threshold=0.5, method="treecode", p=6, theta=0.5,
              ncrit=0, precision="fp32", m2p_min_panels=0, matrix_cores=True,
              stream_narrow=False, pair_operators=False, pair_narrow=False,
              four_wave=False):
    return lspr_op_params(k_far, k_fine, n_k, threshold,
                          LSPR_TREECODE if method == "treecode" else LSPR_DENSE, p, theta, ncrit,
                          _PRECISION[precision], m2p_min_panels,
                          (0 if matrix_cores else LSPR_NO_MATRIX_CORES) |
                          (LSPR_STREAM_NARROW if stream_narrow else 0) |
                          (LSPR_PAIR_OPERATORS if pair_operators else 0) |
                          (LSPR_PAIR_NARROW if pair_narrow else 0) |
                          (LSPR_FOUR_WAVE if four_wave else 0))


def gmres_params(tol=1e-6, restart=60, max_iter=600, precond=1, inner_tol=0.0):
    return lspr_gmres_params(tol, restart, max_iter, precond, inner_tol)


class Geometry:
    """A geometry handle (lspr_geometry_create / lspr_geometry_destroy).

    surfaces: list of (verts, tris); numpy arrays are validated on the host with
    lspr_mesh_validate and uploaded as torch cuda tensors; cuda tensors are used as they are.
    """

    def __init__(self, surfaces, op=None, stream=None, validate=True, **op_kw):
        import torch
        self.op = op if op is not None else op_params(**op_kw)
        dev = []
        host = []
        for v, t in surfaces:
            if isinstance(v, torch.Tensor):
                dv = v.to(dtype=torch.float64).contiguous()
                dt = t.to(dtype=torch.int32).contiguous()
            else:
                host.append((v, t))
                dv = torch.as_tensor(np.ascontiguousarray(v, dtype=np.float64)).cuda()
                dt = torch.as_tensor(np.ascontiguousarray(t, dtype=np.int32)).cuda()
            dev.append((dv, dt))
        if validate and host and len(host) == len(surfaces):
            _check(lspr_mesh_validate(host), "lspr_mesh_validate")
        arr = (lspr_surface * len(dev))()
        for k, (dv, dt) in enumerate(dev):
            arr[k] = lspr_surface(dv.shape[0], dv.data_ptr(), dt.shape[0], dt.data_ptr())
        self._dev = dev
        self.n_surf = len(dev)
        self.n_panels = int(sum(dt.shape[0] for _, dt in dev))
        h = C.c_void_p()
        _check(_lib.lspr_geometry_create(arr, len(dev), C.byref(self.op), _stream_ptr(stream),
                                         C.byref(h)), "lspr_geometry_create")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            _lib.lspr_geometry_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_charges(self, positions, charges, surfaces, stream=None):
        """Point charges inside the surfaces (lspr_geometry_set_charges): positions [n, 3],
        charges [n] (divided by the vacuum permittivity), surfaces [n]; empty removes them."""
        pos = np.ascontiguousarray(np.asarray(positions, dtype=np.float64).reshape(-1, 3))
        q = np.ascontiguousarray(np.asarray(charges, dtype=np.float64).ravel())
        sid = np.ascontiguousarray(np.asarray(surfaces, dtype=np.int32).ravel())
        assert len(pos) == len(q) == len(sid)
        _check(_lib.lspr_geometry_set_charges(
            self.handle, len(q), _dptr(pos), _dptr(q),
            sid.ctypes.data_as(C.POINTER(C.c_int32)), _stream_ptr(stream)),
            "lspr_geometry_set_charges")

    def info(self) -> dict:
        st = lspr_geometry_stats()
        _check(_lib.lspr_geometry_info(self.handle, C.byref(st)), "lspr_geometry_info")
        return {name: getattr(st, name) for name, _ in st._fields_}

    def solve(self, lambdas, eps_medium, eps_surface, e_field=(0.0, 0.0, 1.0), gmres=None,
              stream=None, want_fields=False, allow_noconv=False, **gm_kw):
        """Batched solve; returns a dict of numpy arrays (phi/dphi as torch cuda tensors)."""
        import torch
        lam = np.ascontiguousarray(lambdas, dtype=np.float64).reshape(-1)
        nl = len(lam)
        em, em_p = _c64_array(np.broadcast_to(np.asarray(eps_medium), (nl,)))
        es, es_p = _c64_array(np.asarray(eps_surface).reshape(nl, self.n_surf))
        ef = np.ascontiguousarray(e_field, dtype=np.float64)
        gm = gmres if gmres is not None else gmres_params(**gm_kw)
        phi = dphi = None
        if want_fields:
            phi = torch.zeros((nl, self.n_panels), dtype=torch.complex128, device="cuda")
            dphi = torch.zeros_like(phi)
        ps = np.zeros((nl, 3), np.complex128)
        pt = np.zeros((nl, 3), np.complex128)
        cs = np.zeros(nl)
        ct = np.zeros(nl)
        it = np.zeros(nl, np.int32)
        rr = np.zeros(nl)
        code = _lib.lspr_solve(self.handle, nl, _dptr(lam), em_p, es_p, _dptr(ef), C.byref(gm),
                               _stream_ptr(stream),
                               C.c_void_p(phi.data_ptr() if phi is not None else None),
                               C.c_void_p(dphi.data_ptr() if dphi is not None else None),
                               ps.ctypes.data_as(C.POINTER(lspr_c64)),
                               pt.ctypes.data_as(C.POINTER(lspr_c64)), _dptr(cs), _dptr(ct),
                               it.ctypes.data_as(C.POINTER(C.c_int32)), _dptr(rr))
        _check(code, "lspr_solve", allow=(LSPR_E_NOCONV,) if allow_noconv else ())
        return {"p_sensor": ps, "p_total": pt, "cext_sensor": cs, "cext_total": ct,
                "iters": it, "rel_resid": rr, "phi": phi, "dphi": dphi,
                "converged": code == LSPR_OK}

    def apply(self, x, eps_medium, eps_surface, stream=None, out=None, noalloc=False):
        """y = A x for x a complex128 cuda tensor [n_cols, 2N] (caller's panel order).
        noalloc: through lspr_apply_noalloc (the library allocates no device memory; `out`, a
        complex128 cuda tensor like x, may be given so that the call allocates nothing at all)."""
        import torch
        x = x.to(torch.complex128).contiguous()
        nc = x.shape[0]
        em, em_p = _c64_array(np.broadcast_to(np.asarray(eps_medium), (nc,)))
        es, es_p = _c64_array(np.asarray(eps_surface).reshape(nc, self.n_surf))
        y = torch.empty_like(x) if out is None else out
        if out is not None:
            assert out.dtype == torch.complex128 and out.is_contiguous() and out.shape == x.shape
        fn = _lib.lspr_apply_noalloc if noalloc else _lib.lspr_apply
        name = "lspr_apply_noalloc" if noalloc else "lspr_apply"
        _check(fn(self.handle, nc, em_p, es_p, C.c_void_p(x.data_ptr()),
                  C.c_void_p(y.data_ptr()), _stream_ptr(stream)), name)
        return y

    def rhs(self, eps_medium, eps_surface, e_field=(0.0, 0.0, 1.0), stream=None):
        import torch
        es_arr = np.asarray(eps_surface).reshape(-1, self.n_surf)
        nc = es_arr.shape[0]
        em, em_p = _c64_array(np.broadcast_to(np.asarray(eps_medium), (nc,)))
        es, es_p = _c64_array(es_arr)
        ef = np.ascontiguousarray(e_field, dtype=np.float64)
        b = torch.empty((nc, 2 * self.n_panels), dtype=torch.complex128, device="cuda")
        _check(_lib.lspr_rhs(self.handle, nc, em_p, es_p, _dptr(ef), C.c_void_p(b.data_ptr()),
                             _stream_ptr(stream)), "lspr_rhs")
        return b


# ------------------------------------------------------------------ profiling
_lib.lspr_profile_enable.restype = C.c_int
_lib.lspr_profile_enable.argtypes = [C.c_int32]
_lib.lspr_profile_reset.restype = C.c_int
_lib.lspr_profile_reset.argtypes = []
_lib.lspr_profile_query.restype = C.c_int
_lib.lspr_profile_query_width.restype = C.c_int
_lib.lspr_profile_query_width.argtypes = [C.c_char_p, C.c_int32, C.c_int32,
                                          C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                          C.POINTER(C.c_double), C.POINTER(C.c_double),
                                          C.POINTER(C.c_double)]
_lib.lspr_profile_query.argtypes = [C.c_char_p, C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                    C.POINTER(C.c_double), C.POINTER(C.c_double),
                                    C.POINTER(C.c_double)]


def lspr_profile_enable(on):
    """on: False/0 off, True/1 all launches, 2 far-field launches only."""
    _check(_lib.lspr_profile_enable(int(on)), "lspr_profile_enable")


def lspr_profile_reset():
    _check(_lib.lspr_profile_reset(), "lspr_profile_reset")


def lspr_profile_query(name: str) -> dict:
    ms, fl, by, it = C.c_double(), C.c_double(), C.c_double(), C.c_double()
    n = C.c_int64()
    _check(_lib.lspr_profile_query(name.encode(), C.byref(ms), C.byref(n), C.byref(fl),
                                   C.byref(by), C.byref(it)), "lspr_profile_query")
    return {"total_ms": ms.value, "launches": n.value, "flops": fl.value, "bytes": by.value,
            "items": it.value}


def lspr_profile_query_width(name: str, width_min: int, width_max: int) -> dict:
    """As lspr_profile_query, for the launches of width_min..width_max wavelengths."""
    ms, fl, by, it = C.c_double(), C.c_double(), C.c_double(), C.c_double()
    n = C.c_int64()
    _check(_lib.lspr_profile_query_width(name.encode(), int(width_min), int(width_max),
                                         C.byref(ms), C.byref(n), C.byref(fl), C.byref(by),
                                         C.byref(it)), "lspr_profile_query_width")
    return {"total_ms": ms.value, "launches": n.value, "flops": fl.value, "bytes": by.value,
            "items": it.value}


# ------------------------------------------------------------------ request server
class lspr_server_params(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_int64), ("max_slots", C.c_int32), ("pad", C.c_int32)]


class lspr_request_info(C.Structure):
    _fields_ = [("status", C.c_int32), ("n_lambda", C.c_int32), ("n_panels", C.c_int64),
                ("t_submit", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double),
                ("est_bytes", C.c_int64), ("peak_bytes", C.c_int64), ("error", C.c_char * 256)]


class lspr_server_stats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in (
        "submitted", "completed", "queued", "active", "max_active", "budget_bytes",
        "reserved_bytes", "peak_reserved_bytes", "estimate_violations")]


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args


_P = C.POINTER
_sig("lspr_server_create", C.c_int, [_P(lspr_server_params), _P(C.c_void_p)])
_sig("lspr_server_submit", C.c_int, [C.c_void_p, _P(lspr_surface), C.c_int32, _P(lspr_op_params),
                                     C.c_int32, _P(C.c_double), _P(lspr_c64), _P(lspr_c64),
                                     _P(C.c_double), _P(lspr_gmres_params), _P(C.c_uint64)])
_sig("lspr_server_submit_charges", C.c_int,
     [C.c_void_p, _P(lspr_surface), C.c_int32, _P(lspr_op_params), C.c_int32, _P(C.c_double),
      _P(lspr_c64), _P(lspr_c64), _P(C.c_double), _P(lspr_gmres_params), C.c_int32,
      _P(C.c_double), _P(C.c_double), _P(C.c_int32), _P(C.c_uint64)])
_sig("lspr_server_poll", C.c_int, [C.c_void_p, C.c_uint64, C.c_int32, _P(lspr_request_info),
                                   _P(C.c_double), _P(C.c_double), _P(lspr_c64), _P(lspr_c64),
                                   _P(C.c_int32), _P(C.c_double)])
_sig("lspr_server_stats_get", C.c_int, [C.c_void_p, _P(lspr_server_stats)])
_sig("lspr_server_destroy", C.c_int, [C.c_void_p])
_sig("lspr_request_footprint", C.c_int, [C.c_int64, C.c_int32, C.c_int32, _P(lspr_op_params),
                                         _P(lspr_gmres_params), _P(C.c_int64)])


class lspr_tune_entry(C.Structure):
    _fields_ = [("p", C.c_int32), ("ncrit", C.c_int32), ("theta", C.c_double),
                ("rel_err", C.c_double), ("ms_per_product", C.c_double),
                ("m2p_min_panels", C.c_int32), ("flags", C.c_int32)]


_sig("lspr_autotune", C.c_int, [_P(lspr_surface), C.c_int32, C.c_int32, _P(lspr_c64),
                                 _P(lspr_c64), C.c_double, _P(lspr_op_params),
                                 _P(lspr_tune_entry), C.c_int32, _P(C.c_int32), C.c_void_p])


def lspr_autotune(surfaces, n_cols, eps_medium, eps_surface, max_rel_err=1e-5, op=None,
                  stream=None, **op_kw):
    """Treecode parameters for a mesh (lspr_autotune).  surfaces: list of (verts, tris) torch
    cuda tensors or numpy arrays (uploaded); eps_surface: one value per surface.  Returns
    (op, entries, ok): op the lspr_op_params with the chosen p, theta, ncrit; entries a list of
    dicts (every candidate tried); ok False when no candidate met the bound."""
    import torch
    op = op if op is not None else op_params(**op_kw)
    dev = []
    for v, t in surfaces:
        if isinstance(v, torch.Tensor):
            dev.append((v.to(dtype=torch.float64).contiguous(), t.to(dtype=torch.int32).contiguous()))
        else:
            dev.append((torch.as_tensor(np.ascontiguousarray(v, dtype=np.float64)).cuda(),
                        torch.as_tensor(np.ascontiguousarray(t, dtype=np.int32)).cuda()))
    arr = (lspr_surface * len(dev))()
    for k, (dv, dt) in enumerate(dev):
        arr[k] = lspr_surface(dv.shape[0], dv.data_ptr(), dt.shape[0], dt.data_ptr())
    em = (lspr_c64 * 1)(lspr_c64(complex(eps_medium).real, complex(eps_medium).imag))
    es_list = [complex(e) for e in np.ravel(eps_surface)]
    es = (lspr_c64 * len(es_list))(*[lspr_c64(e.real, e.imag) for e in es_list])
    cap = 256
    ent = (lspr_tune_entry * cap)()
    n = C.c_int32()
    code = _lib.lspr_autotune(arr, len(dev), int(n_cols), em, es, float(max_rel_err),
                              C.byref(op), ent, cap, C.byref(n), _stream_ptr(stream))
    _check(code, "lspr_autotune", allow=(LSPR_E_NOCONV,))
    entries = [{name: getattr(ent[k], name) for name, _ in lspr_tune_entry._fields_}
               for k in range(min(n.value, cap))]
    return op, entries, code == LSPR_OK


def lspr_request_footprint(n_panels, n_surf, n_lambda, op, gm) -> int:
    out = C.c_int64()
    _check(_lib.lspr_request_footprint(n_panels, n_surf, n_lambda, C.byref(op), C.byref(gm),
                                       C.byref(out)), "lspr_request_footprint")
    return out.value


class Server:
    """Request server (lspr_server_*): continuous batching of solve requests on the current
    device.  Meshes are host arrays; submit() copies them and returns a ticket at once."""

    def __init__(self, hbm_budget_bytes=0, max_slots=4):
        h = C.c_void_p()
        prm = lspr_server_params(int(hbm_budget_bytes), int(max_slots), 0)
        _check(_lib.lspr_server_create(C.byref(prm), C.byref(h)), "lspr_server_create")
        self.handle = h
        self._nl = {}

    def submit(self, surfaces, lambdas, eps_medium, eps_surface, e_field=(0.0, 0.0, 1.0),
               op=None, gmres=None, charges=None) -> int:
        """Queues one request; charges = (positions [n, 3], charges [n], surfaces [n]) or None
        (lspr_server_submit_charges / lspr_server_submit)."""
        lam = np.ascontiguousarray(lambdas, dtype=np.float64).reshape(-1)
        nl = len(lam)
        ns = len(surfaces)
        em, em_p = _c64_array(np.broadcast_to(np.asarray(eps_medium), (nl,)))
        es, es_p = _c64_array(np.asarray(eps_surface).reshape(nl, ns))
        ef = np.ascontiguousarray(e_field, dtype=np.float64)
        keep = []
        arr = (lspr_surface * ns)()
        for k, (v, t) in enumerate(surfaces):
            v = np.ascontiguousarray(v, dtype=np.float64)
            t = np.ascontiguousarray(t, dtype=np.int32)
            keep += [v, t]
            arr[k] = lspr_surface(len(v), v.ctypes.data, len(t), t.ctypes.data)
        op = op if op is not None else op_params()
        gm = gmres if gmres is not None else gmres_params()
        tk = C.c_uint64()
        if charges is None:
            _check(_lib.lspr_server_submit(self.handle, arr, ns, C.byref(op), nl, _dptr(lam),
                                           em_p, es_p, _dptr(ef), C.byref(gm), C.byref(tk)),
                   "lspr_server_submit")
        else:
            pos = np.ascontiguousarray(np.asarray(charges[0], dtype=np.float64).reshape(-1, 3))
            q = np.ascontiguousarray(np.asarray(charges[1], dtype=np.float64).ravel())
            sid = np.ascontiguousarray(np.asarray(charges[2], dtype=np.int32).ravel())
            assert len(pos) == len(q) == len(sid)
            _check(_lib.lspr_server_submit_charges(
                self.handle, arr, ns, C.byref(op), nl, _dptr(lam), em_p, es_p, _dptr(ef),
                C.byref(gm), len(q), _dptr(pos), _dptr(q),
                sid.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(tk)),
                "lspr_server_submit_charges")
        self._nl[tk.value] = nl
        return tk.value

    def poll(self, ticket: int, wait: bool = False):
        """None while the request runs (wait=False); else a dict with its results."""
        nl = self._nl.get(ticket, 0)  # unknown tickets are reported by the library
        info = lspr_request_info()
        cs, ct, rr = np.zeros(nl), np.zeros(nl), np.zeros(nl)
        ps = np.zeros((nl, 3), np.complex128)
        pt = np.zeros((nl, 3), np.complex128)
        it = np.zeros(nl, np.int32)
        code = _lib.lspr_server_poll(self.handle, ticket, 1 if wait else 0, C.byref(info),
                                     _dptr(cs), _dptr(ct), ps.ctypes.data_as(_P(lspr_c64)),
                                     pt.ctypes.data_as(_P(lspr_c64)),
                                     it.ctypes.data_as(_P(C.c_int32)), _dptr(rr))
        if code == LSPR_E_BUSY:
            return None
        _check(code, "lspr_server_poll")
        self._nl.pop(ticket, None)
        out = {name: getattr(info, name) for name, _ in info._fields_}
        out["error"] = info.error.decode(errors="replace")
        out.update(cext_sensor=cs, cext_total=ct, p_sensor=ps, p_total=pt, iters=it,
                   rel_resid=rr, latency_s=info.t_done - info.t_submit)
        return out

    def stats(self) -> dict:
        st = lspr_server_stats()
        _check(_lib.lspr_server_stats_get(self.handle, C.byref(st)), "lspr_server_stats_get")
        return {name: getattr(st, name) for name, _ in st._fields_}

    def close(self):
        if getattr(self, "handle", None):
            _check(_lib.lspr_server_destroy(self.handle), "lspr_server_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
