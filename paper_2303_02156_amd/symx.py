"""ctypes binding of libsymx.so (argument marshalling only).

The functions below carry the C-ABI names of include/symx.h and forward to the
library; every computation runs in the library's HIP kernels.  PyTorch
provides device memory (float64 CUDA/HIP tensors) and the stream.  The library
must be built (paper_2303_02156_amd.build); importing it on a machine without
it raises, there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(_PKG, "libsymx.so")

SYMX_OK = 0
STATUS = {0: "OK", 1: "INVALID_ARG", 2: "OUT_OF_MEMORY", 3: "DEVICE", 4: "NONFINITE",
          5: "NOT_CONVERGED", 6: "LINE_SEARCH", 7: "BUDGET", 8: "PENDING"}
SYMX_PENDING = 8
SYMX_F64, SYMX_F32, SYMX_F32_REFINED = 0, 1, 2
SYMX_CONTACT_COMPACT, SYMX_CONTACT_BRANCH = 0, 1
SYMX_SNH_TET4, SYMX_STVK_TRI3, SYMX_HINGE4 = 0, 1, 2
SYMX_NH_TET4, SYMX_STVK_TET4, SYMX_FCR_TET4, SYMX_ARAP_TET4 = 3, 4, 5, 6
SYMX_EVAL_E, SYMX_EVAL_GRAD, SYMX_EVAL_HESS, SYMX_PROJECT_PSD, SYMX_DIRICHLET = 1, 2, 4, 8, 16
SYMX_PROJECT_FILTER = 32
SYMX_SNH_TET10, SYMX_SNH_TET20 = 7, 8


class EnergyDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_elem", C.c_int64), ("conn", C.c_void_p),
                ("young", C.c_void_p), ("young_const", C.c_double), ("poisson", C.c_double),
                ("thickness", C.c_double), ("bend_kb", C.c_double), ("density", C.c_double)]


class MeshDesc(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("x_rest", C.c_void_p), ("n_energies", C.c_int32),
                ("energies", C.POINTER(EnergyDesc)), ("fixed", C.c_void_p),
                ("hip_stream", C.c_void_p)]


class BsrView(C.Structure):
    _fields_ = [("n_block_rows", C.c_int64), ("nnzb", C.c_int64), ("row_ptr", C.c_void_p),
                ("col_idx", C.c_void_p), ("values", C.c_void_p), ("precision", C.c_int32)]


class MeshInfo(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("nnzb", C.c_int64), ("n_incidences", C.c_int64),
                ("n_batches", C.c_int64), ("n_elem", C.c_int64 * 4), ("n_energies", C.c_int32),
                ("max_row_blocks", C.c_int32), ("total_mass", C.c_double)]


class StepParams(C.Structure):
    _fields_ = [("dt", C.c_double), ("gravity", C.c_double * 3), ("newton_rtol", C.c_double),
                ("max_newton", C.c_int32), ("max_pcg", C.c_int32), ("project", C.c_int32),
                ("precision", C.c_int32), ("max_halvings", C.c_int32),
                ("regrow_after", C.c_int32), ("max_refine", C.c_int32),
                ("forcing_max", C.c_double)]


class StepReport(C.Structure):
    _fields_ = [("status", C.c_int32), ("newton_iters", C.c_int32), ("pcg_iters", C.c_int32),
                ("ls_backtracks", C.c_int32), ("dt_halvings", C.c_int32),
                ("refinements", C.c_int32), ("dt_used", C.c_double), ("residual0", C.c_double),
                ("residual", C.c_double), ("energy", C.c_double), ("ms_assemble", C.c_double),
                ("ms_pcg", C.c_double), ("ms_linesearch", C.c_double), ("ms_total", C.c_double),
                ("lin_residual", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class ServerStats(C.Structure):
    _fields_ = [("budget_bytes", C.c_uint64), ("in_use_bytes", C.c_uint64),
                ("peak_bytes", C.c_uint64), ("pattern_cache_bytes", C.c_uint64),
                ("queued", C.c_int64), ("completed", C.c_int64), ("pattern_hits", C.c_int64),
                ("pattern_misses", C.c_int64), ("pcg_batches", C.c_int64),
                ("pcg_chunks", C.c_int64), ("active", C.c_int32), ("peak_active", C.c_int32),
                ("max_slots", C.c_int32), ("peak_device_bytes", C.c_uint64)]


EXPORTS = {
    "symx_step_params_default": (None, [C.POINTER(StepParams)]),
    "symx_mesh_create": (C.c_int, [C.POINTER(MeshDesc), C.POINTER(C.c_void_p)]),
    "symx_mesh_destroy": (C.c_int, [C.c_void_p]),
    "symx_mesh_get_info": (C.c_int, [C.c_void_p, C.POINTER(MeshInfo)]),
    "symx_mesh_get_pattern": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "symx_mesh_get_masses": (C.c_int, [C.c_void_p, C.c_void_p]),
    "symx_eval_derivatives": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_uint32, C.c_int32,
                                        C.c_void_p, C.c_void_p, C.c_void_p]),
    "symx_assemble_bsr": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_uint32,
                                    C.c_int32, C.POINTER(C.c_double), C.c_void_p,
                                    C.POINTER(BsrView)]),
    "symx_assemble_bsr_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                                            C.c_uint32, C.c_int32, C.POINTER(C.c_double),
                                            C.c_void_p, C.c_void_p]),
    "symx_newton_step": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(StepParams),
                                   C.POINTER(StepReport)]),
    "symx_mesh_update_rotations": (C.c_int, [C.c_void_p, C.c_void_p]),
    "symx_mesh_set_contacts": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_double,
                                         C.c_double]),
    "symx_mesh_get_contact_bsr": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(BsrView)]),
    "symx_mesh_set_contact_mode": (C.c_int, [C.c_void_p, C.c_int32]),
    "symx_mesh_set_dynamic_elements": (C.c_int, [C.c_void_p, C.POINTER(EnergyDesc)]),
    "symx_mesh_set_profiling": (C.c_int, [C.c_void_p, C.c_int32]),
    "symx_mesh_get_kernel_time": (C.c_int, [C.c_void_p, C.c_char_p, C.c_double,
                                            C.POINTER(C.c_int64), C.POINTER(C.c_double)]),
    "symx_mesh_kernel_names": (C.c_int, [C.c_void_p, C.c_char_p, C.c_int64]),
    "symx_server_create": (C.c_int, [C.c_uint64, C.c_int32, C.POINTER(C.c_void_p)]),
    "symx_server_submit": (C.c_int, [C.c_void_p, C.POINTER(MeshDesc), C.c_void_p, C.c_void_p,
                                     C.POINTER(StepParams), C.POINTER(C.c_int64)]),
    "symx_server_poll": (C.c_int, [C.c_void_p, C.c_int64, C.c_int32, C.c_void_p, C.c_void_p,
                                   C.POINTER(StepReport), C.c_void_p]),
    "symx_server_get_stats": (C.c_int, [C.c_void_p, C.POINTER(ServerStats)]),
    "symx_server_destroy": (C.c_int, [C.c_void_p]),
    "symx_server_estimate_bytes": (C.c_int, [C.POINTER(MeshDesc), C.c_int32,
                                             C.POINTER(C.c_uint64)]),
    "symx_status_string": (C.c_char_p, [C.c_int]),
    "symx_last_error": (C.c_char_p, []),
}

_lib = None


def load():
    """Load libsymx.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise RuntimeError(f"libsymx.so not found at {LIBPATH}; run __graft_entry__.build()")
        lib = C.CDLL(LIBPATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class SymxError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = load().symx_last_error().decode()
        super().__init__(f"{where}: {STATUS.get(status, status)}: {msg}")


def _check(st, where):
    if st != SYMX_OK:
        raise SymxError(st, where)


# --- the C-ABI entry points, same names ------------------------------------
def symx_mesh_create(desc):
    h = C.c_void_p()
    _check(load().symx_mesh_create(C.byref(desc), C.byref(h)), "symx_mesh_create")
    return h


def symx_mesh_destroy(h):
    _check(load().symx_mesh_destroy(h), "symx_mesh_destroy")


def symx_mesh_get_info(h):
    info = MeshInfo()
    _check(load().symx_mesh_get_info(h, C.byref(info)), "symx_mesh_get_info")
    return info


def symx_mesh_get_pattern(h, row_ptr, col_idx, scatter_map):
    _check(load().symx_mesh_get_pattern(h, row_ptr, col_idx, scatter_map), "symx_mesh_get_pattern")


def symx_mesh_get_masses(h, mass_host):
    _check(load().symx_mesh_get_masses(h, mass_host), "symx_mesh_get_masses")


def symx_eval_derivatives(h, set_index, x_dev, flags, precision, e_dev, g_dev, H_dev):
    _check(load().symx_eval_derivatives(h, set_index, x_dev, flags, precision, e_dev, g_dev, H_dev),
           "symx_eval_derivatives")


def symx_assemble_bsr(h, x_dev, xt_dev, dt, flags, precision, grad_dev):
    E = C.c_double(0.0)
    view = BsrView()
    _check(load().symx_assemble_bsr(h, x_dev, xt_dev, dt, flags, precision, C.byref(E), grad_dev,
                                    C.byref(view)), "symx_assemble_bsr")
    return E.value, view


def symx_assemble_bsr_noalloc(h, x_dev, xt_dev, dt, flags, precision, grad_dev, values_dev):
    """Returns (status, energy): the allocation-free assembly into values_dev."""
    E = C.c_double(0.0)
    st = load().symx_assemble_bsr_noalloc(h, x_dev, xt_dev, dt, flags, precision, C.byref(E),
                                          grad_dev, values_dev)
    return st, E.value


def symx_newton_step(h, x_dev, v_dev, params):
    rep = StepReport()
    st = load().symx_newton_step(h, x_dev, v_dev, C.byref(params), C.byref(rep))
    return st, rep


def symx_mesh_update_rotations(h, x_dev):
    _check(load().symx_mesh_update_rotations(h, x_dev), "symx_mesh_update_rotations")


def symx_mesh_set_contacts(h, tuples_host, kc, dhat):
    t = np.ascontiguousarray(tuples_host, dtype=np.int32).reshape(-1, 4)
    _check(load().symx_mesh_set_contacts(h, t.shape[0], t.ctypes.data if t.size else None, kc, dhat),
           "symx_mesh_set_contacts")


def symx_mesh_get_contact_bsr(h, precision):
    view = BsrView()
    _check(load().symx_mesh_get_contact_bsr(h, precision, C.byref(view)),
           "symx_mesh_get_contact_bsr")
    return view


def symx_mesh_set_profiling(h, enable):
    _check(load().symx_mesh_set_profiling(h, int(enable)), "symx_mesh_set_profiling")


def symx_mesh_get_kernel_time(h, name, min_ms=0.0):
    n = C.c_int64(0)
    ms = C.c_double(0.0)
    _check(load().symx_mesh_get_kernel_time(h, name.encode(), min_ms, C.byref(n), C.byref(ms)),
           "symx_mesh_get_kernel_time")
    return n.value, ms.value


def symx_mesh_kernel_names(h):
    buf = C.create_string_buffer(4096)
    _check(load().symx_mesh_kernel_names(h, buf, 4096), "symx_mesh_kernel_names")
    v = buf.value.decode()
    return v.split(",") if v else []


def symx_step_params_default():
    p = StepParams()
    load().symx_step_params_default(C.byref(p))
    return p


def symx_server_create(budget_bytes, max_slots):
    h = C.c_void_p()
    _check(load().symx_server_create(int(budget_bytes), int(max_slots), C.byref(h)),
           "symx_server_create")
    return h


def symx_server_submit(h, desc, x_host, v_host, params):
    t = C.c_int64(0)
    _check(load().symx_server_submit(h, C.byref(desc), x_host.ctypes.data, v_host.ctypes.data,
                                     C.byref(params), C.byref(t)), "symx_server_submit")
    return t.value


def symx_server_poll(h, ticket, wait, x_out=None, v_out=None):
    rep = StepReport()
    times = np.zeros(5)
    st = load().symx_server_poll(h, ticket, int(wait),
                                 None if x_out is None else x_out.ctypes.data,
                                 None if v_out is None else v_out.ctypes.data,
                                 C.byref(rep), times.ctypes.data)
    return st, rep, times


def symx_server_get_stats(h):
    s = ServerStats()
    _check(load().symx_server_get_stats(h, C.byref(s)), "symx_server_get_stats")
    return s


def symx_server_estimate_bytes(desc, precision):
    b = C.c_uint64(0)
    _check(load().symx_server_estimate_bytes(C.byref(desc), int(precision), C.byref(b)),
           "symx_server_estimate_bytes")
    return b.value


def symx_server_destroy(h):
    _check(load().symx_server_destroy(h), "symx_server_destroy")


# --- convenience wrapper around a scene (marshalling only) -------------------
def _ptr(a):
    return None if a is None else a.ctypes.data


def scene_desc(scene, stream_handle=None):
    """Build a MeshDesc for a scenegen.Scene-like object.  Returns (desc, keep):
    `keep` holds the arrays the descriptor points to and must outlive its use."""
    keep = []
    descs = (EnergyDesc * len(scene.energies))()
    for i, es in enumerate(scene.energies):
        conn = np.ascontiguousarray(es.conn, dtype=np.int32)
        young = None
        if es.young_per_elem is not None:
            young = np.ascontiguousarray(es.young_per_elem, dtype=np.float64)
        keep += [conn, young]
        descs[i] = EnergyDesc(es.kind, conn.shape[0], _ptr(conn), _ptr(young), float(es.young),
                              float(es.poisson), float(es.thickness), float(es.bend_kb),
                              float(es.density))
    X = np.ascontiguousarray(scene.X, dtype=np.float64)
    fixed = np.ascontiguousarray(scene.fixed, dtype=np.uint8)
    keep += [descs, X, fixed]
    desc = MeshDesc(scene.n_nodes, _ptr(X), len(scene.energies), descs, _ptr(fixed),
                    C.c_void_p(stream_handle or 0))
    return desc, keep


class Mesh:
    """Owns one library mesh built from a scenegen.Scene-like object."""

    def __init__(self, scene, stream=None):
        import torch
        self.torch = torch
        self.N = scene.n_nodes
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        desc, keep = scene_desc(scene, stream.cuda_stream)
        self.handle = symx_mesh_create(desc)
        self.info = symx_mesh_get_info(self.handle)
        self.kinds = [es.kind for es in scene.energies]
        self.n_elem = [es.conn.shape[0] for es in scene.energies]
        self.nodes_per_elem = [es.conn.shape[1] for es in scene.energies]

    def close(self):
        if getattr(self, "handle", None):
            symx_mesh_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # host-side pattern
    def pattern(self):
        N, nnzb = self.info.n_nodes, self.info.nnzb
        rp = np.zeros(N + 1, dtype=np.int32)
        ci = np.zeros(nnzb, dtype=np.int32)
        total = sum(n * k * k for n, k in zip(self.n_elem, self.nodes_per_elem))
        sm = np.zeros(max(total, 1), dtype=np.int32)
        symx_mesh_get_pattern(self.handle, rp.ctypes.data, ci.ctypes.data, sm.ctypes.data)
        maps, off = [], 0
        for n, k in zip(self.n_elem, self.nodes_per_elem):
            maps.append(sm[off:off + n * k * k].reshape(n, k, k))
            off += n * k * k
        return rp, ci, maps

    def masses(self):
        m = np.zeros(self.N)
        symx_mesh_get_masses(self.handle, m.ctypes.data)
        return m

    def _dev(self, a):
        t = self.torch
        if isinstance(a, t.Tensor):
            assert a.is_cuda and a.dtype == t.float64 and a.is_contiguous()
            return a
        return t.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")

    def eval_derivatives(self, set_index, x, flags=SYMX_EVAL_E | SYMX_EVAL_GRAD | SYMX_EVAL_HESS,
                         precision=SYMX_F64):
        t = self.torch
        xd = self._dev(x)
        n = self.n_elem[set_index]
        D = 3 * self.nodes_per_elem[set_index]
        dtype = t.float64 if precision == SYMX_F64 else t.float32
        E = t.empty(max(n, 1), dtype=dtype, device="cuda")
        g = t.empty((max(n, 1), D), dtype=dtype, device="cuda")
        H = t.empty((max(n, 1), D, D), dtype=dtype, device="cuda")
        symx_eval_derivatives(self.handle, set_index, xd.data_ptr(), flags, precision, E.data_ptr(),
                              g.data_ptr(), H.data_ptr())
        return E[:n], g[:n], H[:n]

    def assemble(self, x, x_tilde=None, dt=0.0, flags=SYMX_EVAL_E | SYMX_EVAL_GRAD | SYMX_EVAL_HESS,
                 precision=SYMX_F64, grad_out=None):
        """Returns (energy, gradient tensor (N,3) float64, values tensor (9, nnzb) or None)."""
        t = self.torch
        xd = self._dev(x)
        xt = self._dev(x_tilde) if x_tilde is not None else None
        g = grad_out if grad_out is not None else t.empty((self.N, 3), dtype=t.float64, device="cuda")
        E, view = symx_assemble_bsr(self.handle, xd.data_ptr(), None if xt is None else xt.data_ptr(),
                                    dt, flags, precision, g.data_ptr())
        vals = None
        if flags & SYMX_EVAL_HESS:
            dtype = t.float64 if precision == SYMX_F64 else t.float32
            vals = t.empty((9, self.info.nnzb), dtype=dtype, device="cuda")
            _device_copy(vals.data_ptr(), view.values, vals.numel() * vals.element_size())
        return E, g, vals

    def set_contacts(self, tuples, kc, dhat):
        """Candidate contacts (n x 4: point, triangle) of the barrier."""
        symx_mesh_set_contacts(self.handle, tuples, kc, dhat)

    def set_dynamic_elements(self, es):
        """Replace the dynamic element set by the scenegen.EnergySet `es` (None
        or an empty set removes it)."""
        n = 0 if es is None else int(es.conn.shape[0])
        conn = np.ascontiguousarray(np.zeros((0, 4)) if es is None else es.conn, dtype=np.int32)
        young = None
        if es is not None and es.young_per_elem is not None:
            young = np.ascontiguousarray(es.young_per_elem, dtype=np.float64)
        d = EnergyDesc(0 if es is None else es.kind, n, _ptr(conn), _ptr(young),
                       0.0 if es is None else float(es.young),
                       0.0 if es is None else float(es.poisson),
                       0.0 if es is None else float(es.thickness),
                       0.0 if es is None else float(es.bend_kb),
                       0.0 if es is None else float(es.density))
        _check(load().symx_mesh_set_dynamic_elements(self.handle, C.byref(d)),
               "symx_mesh_set_dynamic_elements")

    def set_contact_mode(self, mode):
        _check(load().symx_mesh_set_contact_mode(self.handle, mode), "symx_mesh_set_contact_mode")

    def contact_bsr(self, precision=SYMX_F64):
        """Host copies (row_ptr, col_idx, values (nnzb, 3, 3) float64) of the
        contact matrix of the last assembly."""
        t = self.torch
        v = symx_mesh_get_contact_bsr(self.handle, precision)
        if v.nnzb == 0:
            return np.zeros(self.N + 1, np.int32), np.zeros(0, np.int32), np.zeros((0, 3, 3))
        rp = t.empty(self.N + 1, dtype=t.int32, device="cuda")
        ci = t.empty(v.nnzb, dtype=t.int32, device="cuda")
        dtype = t.float64 if precision == SYMX_F64 else t.float32
        vals = t.empty((9, v.nnzb), dtype=dtype, device="cuda")
        _device_copy(rp.data_ptr(), v.row_ptr, rp.numel() * 4)
        _device_copy(ci.data_ptr(), v.col_idx, ci.numel() * 4)
        _device_copy(vals.data_ptr(), v.values, vals.numel() * vals.element_size())
        return (rp.cpu().numpy(), ci.cpu().numpy(),
                vals.cpu().numpy().astype(np.float64).T.reshape(-1, 3, 3))

    def update_rotations(self, x):
        """Lagged rotations of the co-rotational and ARAP sets taken at x."""
        symx_mesh_update_rotations(self.handle, self._dev(x).data_ptr())

    def profile(self, enable=True):
        symx_mesh_set_profiling(self.handle, enable)

    def kernel_times(self, min_ms=0.0):
        """{kernel name: (launches, total device ms)} since profiling was enabled,
        counting launches of at least min_ms."""
        return {n: symx_mesh_get_kernel_time(self.handle, n, min_ms)
                for n in symx_mesh_kernel_names(self.handle)}

    def newton_step(self, x, v, params):
        st, rep = symx_newton_step(self.handle, x.data_ptr(), v.data_ptr(), params)
        return st, rep


_hip = None


def _device_copy(dst, src, nbytes):
    """Device-to-device copy of a mesh-owned buffer into a caller tensor."""
    global _hip
    if _hip is None:
        _hip = C.CDLL("libamdhip64.so")
        _hip.hipMemcpy.restype = C.c_int
        _hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
    st = _hip.hipMemcpy(C.c_void_p(dst), C.c_void_p(src), C.c_size_t(nbytes), 3)
    if st != 0:
        raise RuntimeError(f"hipMemcpy failed with {st}")


def step_params(**kw):
    p = symx_step_params_default()
    for k, v in kw.items():
        if k == "gravity":
            for i in range(3):
                p.gravity[i] = v[i]
        else:
            setattr(p, k, v)
    return p
