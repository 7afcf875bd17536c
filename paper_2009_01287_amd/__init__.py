"""MI355X hp-DG subspace-correction solver: Python binding of libhpdg.so.

The binding only marshals arguments; every step of setup and solve runs in
the native library (host setup in C++, operator and preconditioner
applications in HIP kernels). Import fails loudly if the library has not
been built (python -m paper_2009_01287_amd.build).

Entry points mirror include/hpdg.h: Mesh (hpdg_setup_mesh), Operator
(hpdg_setup_operator) with rhs, apply_A, apply_B, pcg_solve and export.
Vectors are torch tensors on the GPU (float64, contiguous); their data
pointers and torch's current stream are handed to the library.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhpdg.so")

STATUS = {0: "OK", -1: "INVALID", -2: "NOMEM", -3: "HIP", -4: "NOT_SPD", -5: "NOT_CONVERGED",
          -6: "UNSUPPORTED", -7: "BUSY"}


class HpdgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"hpdg {STATUS.get(code, code)}: {msg}")
        self.code = code


class Opts(C.Structure):
    _fields_ = [("form", C.c_int), ("penalty_rule", C.c_int), ("eta", C.c_double),
                ("prec_fp32", C.c_int), ("remark_relax", C.c_int), ("jb_only", C.c_int),
                ("max_block", C.c_int), ("max_nrhs", C.c_int), ("host_only", C.c_int), ("no_prec", C.c_int),
                ("graph", C.c_int), ("setup_threads", C.c_int), ("auto_cycle", C.c_int)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int), ("converged", C.c_int), ("rel_res", C.c_double),
                ("true_rel_res", C.c_double), ("lambda_min", C.c_double), ("lambda_max", C.c_double),
                ("cond_est", C.c_double), ("t_solve_s", C.c_double), ("t_setup_s", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


SYMBOLS = ["hpdg_last_error", "hpdg_setup_mesh", "hpdg_mesh_info", "hpdg_mesh_destroy",
           "hpdg_setup_operator", "hpdg_operator_destroy", "hpdg_rhs", "hpdg_apply_A",
           "hpdg_apply_B", "hpdg_apply_B_noalloc", "hpdg_pcg_solve", "hpdg_export", "hpdg_operator_upload",
           "hpdg_operator_device_bytes", "hpdg_batch_create", "hpdg_batch_destroy", "hpdg_batch_admit",
           "hpdg_batch_step", "hpdg_batch_poll", "hpdg_operator_tune"]

_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with python -m paper_2009_01287_amd.build")
    # torch ships its own HIP runtime with the same soname as the system one;
    # loading torch first makes the library bind to that single runtime
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    vp, i32p, f64p = C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_double)
    L.hpdg_last_error.restype = C.c_char_p
    L.hpdg_setup_mesh.argtypes = [C.c_int, C.c_int, C.c_int64, i32p, i32p, i32p, f64p, C.POINTER(vp)]
    L.hpdg_mesh_info.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int)]
    L.hpdg_mesh_destroy.argtypes = [vp]
    L.hpdg_mesh_destroy.restype = None
    L.hpdg_setup_operator.argtypes = [vp, C.POINTER(Opts), vp, C.POINTER(vp)]
    L.hpdg_operator_destroy.argtypes = [vp]
    L.hpdg_operator_destroy.restype = None
    for f in ("hpdg_rhs", "hpdg_apply_A", "hpdg_apply_B", "hpdg_apply_B_noalloc"):
        getattr(L, f).argtypes = [vp, vp, vp, C.c_int, vp]
    L.hpdg_pcg_solve.argtypes = [vp, vp, vp, C.c_int, C.c_double, C.c_int, vp, C.POINTER(SolveInfo)]
    L.hpdg_export.argtypes = [vp, C.c_int, vp, C.POINTER(C.c_size_t)]
    L.hpdg_operator_upload.argtypes = [vp, vp]
    L.hpdg_operator_device_bytes.argtypes = [vp, C.POINTER(C.c_int64)]
    L.hpdg_operator_tune.argtypes = [vp, vp, C.POINTER(C.c_int64), C.c_int, C.POINTER(C.c_int)]
    L.hpdg_batch_create.argtypes = [C.c_int, C.POINTER(vp)]
    L.hpdg_batch_destroy.argtypes = [vp]
    L.hpdg_batch_destroy.restype = None
    L.hpdg_batch_admit.argtypes = [vp, vp, vp, vp, C.c_double, C.c_int, C.c_int64]
    L.hpdg_batch_step.argtypes = [vp, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]
    L.hpdg_batch_poll.argtypes = [vp, C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_int), C.POINTER(SolveInfo),
                                  C.POINTER(C.c_int)]
    _lib = L
    return L


def _check(code):
    if code != 0:
        raise HpdgError(code, lib().hpdg_last_error().decode())


def _stream(stream):
    if stream is not None:
        return C.c_void_p(stream)
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, what):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{what}: expected a contiguous float64 CUDA tensor")
    return C.c_void_p(t.data_ptr())


class Mesh:
    """hpdg_setup_mesh on a mesh dict (dim, n_base, level, anchor, degree,
    kcoef) as produced by hpinputs."""

    def __init__(self, m):
        L = lib()
        self.dim = int(m["dim"])
        lev = np.ascontiguousarray(m["level"], dtype=np.int32)
        anc = np.ascontiguousarray(m["anchor"], dtype=np.int32).reshape(-1)
        deg = np.ascontiguousarray(m["degree"], dtype=np.int32)
        kc = np.ascontiguousarray(m["kcoef"], dtype=np.float64)
        h = C.c_void_p()
        _check(L.hpdg_setup_mesh(self.dim, int(m["n_base"]), len(lev),
                                 lev.ctypes.data_as(C.POINTER(C.c_int32)),
                                 anc.ctypes.data_as(C.POINTER(C.c_int32)),
                                 deg.ctypes.data_as(C.POINTER(C.c_int32)),
                                 kc.ctypes.data_as(C.POINTER(C.c_double)), C.byref(h)))
        self.h = h
        nd, nf, j = C.c_int64(), C.c_int64(), C.c_int()
        _check(L.hpdg_mesh_info(h, C.byref(nd), C.byref(nf), C.byref(j)))
        self.ndof, self.nface, self.max_level_jump = nd.value, nf.value, j.value

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.hpdg_mesh_destroy(self.h)
            self.h = None


class Operator:
    """hpdg_setup_operator. form: 'sipg' or 'br2'."""

    def __init__(self, mesh: Mesh, form="sipg", penalty_rule=0, eta=1.0, prec_fp32=False,
                 remark_relax=False, jb_only=False, max_block=0, max_nrhs=1, host_only=False,
                 no_prec=False, graph=False, setup_threads=0, auto_cycle=False, stream=None):
        L = lib()
        self.mesh = mesh
        self.ndof = mesh.ndof
        self.max_nrhs = max_nrhs
        o = Opts(0 if form == "sipg" else 1 if form == "br2" else -1, penalty_rule, float(eta),
                 int(prec_fp32), int(remark_relax), int(jb_only), int(max_block), int(max_nrhs),
                 int(host_only), int(no_prec), int(graph), int(setup_threads), int(auto_cycle))
        h = C.c_void_p()
        _check(L.hpdg_setup_operator(mesh.h, C.byref(o), C.c_void_p(0) if host_only else _stream(stream),
                                     C.byref(h)))
        self.h = h

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.hpdg_operator_destroy(self.h)
            self.h = None

    def _vec(self, name, a, b, nrhs, stream):
        _check(getattr(lib(), name)(self.h, _ptr(a, "input"), _ptr(b, "output"), int(nrhs), _stream(stream)))

    def rhs(self, f, b, nrhs=1, stream=None):
        self._vec("hpdg_rhs", f, b, nrhs, stream)

    def apply_A(self, x, y, nrhs=1, stream=None):
        self._vec("hpdg_apply_A", x, y, nrhs, stream)

    def apply_B(self, r, z, nrhs=1, stream=None):
        self._vec("hpdg_apply_B", r, z, nrhs, stream)

    def apply_B_noalloc(self, r, z, nrhs=1, stream=None):
        """hpdg_apply_B_noalloc: z = B r with the work vectors in the library's
        static scratch array (no device allocation)."""
        self._vec("hpdg_apply_B_noalloc", r, z, nrhs, stream)

    def pcg_solve(self, b, x, nrhs=1, rtol=1e-8, maxit=1000, stream=None, raise_on_error=True):
        info = (SolveInfo * nrhs)()
        code = lib().hpdg_pcg_solve(self.h, _ptr(b, "b"), _ptr(x, "x"), int(nrhs), float(rtol), int(maxit),
                                    _stream(stream), info)
        out = [i.as_dict() for i in info]
        if code != 0 and raise_on_error:
            raise HpdgError(code, lib().hpdg_last_error().decode())
        return (code, out) if not raise_on_error else out

    def upload(self, stream=None):
        """hpdg_operator_upload: device copy of a host_only operator."""
        _check(lib().hpdg_operator_upload(self.h, _stream(stream)))

    def tune(self, stream=None):
        """hpdg_operator_tune: per-matrix row binning picked by timing; returns
        one dict per matrix."""
        cap = 64
        rep = (C.c_int64 * (8 * cap))()
        n = C.c_int()
        _check(lib().hpdg_operator_tune(self.h, _stream(stream), rep, cap, C.byref(n)))
        kinds = {0: "A", 1: "R", 2: "P", 3: "PT", 4: "elem", 5: "vcycle_fused", 6: "elem_rhs_group", 7: "front_block_lanes", 8: "vcycle_dense_tail", 10: "elem_order", 11: "B_fork"}
        out = []
        for i in range(n.value):
            r = rep[8 * i:8 * i + 8]
            out.append({"matrix": kinds[int(r[0])], "level": int(r[1]), "rows": int(r[2]), "nnz": int(r[3]),
                        "longrow": int(r[4]), "lanes": int(r[5]), "ns_default": int(r[6]), "ns_tuned": int(r[7])})
        return out

    def device_bytes(self):
        b = C.c_int64(0)
        _check(lib().hpdg_operator_device_bytes(self.h, C.byref(b)))
        return b.value

    def export(self, what):
        n = C.c_size_t(0)
        _check(lib().hpdg_export(self.h, int(what), None, C.byref(n)))
        buf = np.zeros(n.value, dtype=np.uint8)
        _check(lib().hpdg_export(self.h, int(what), buf.ctypes.data_as(C.c_void_p), C.byref(n)))
        return buf

    # typed views of the exports
    def diag(self):
        return self.export(0).view(np.float64)

    def labels(self):
        return self.export(1).view(np.int8)

    @staticmethod
    def _csr(buf):
        import scipy.sparse as sp
        hdr = buf[:24].view(np.int64)
        nr, nc, nnz = (int(v) for v in hdr)
        o = 24
        ptr = buf[o:o + 8 * (nr + 1)].view(np.int64)
        o += 8 * (nr + 1)
        idx = buf[o:o + 4 * nnz].view(np.int32)
        o += 4 * nnz
        val = buf[o:o + 8 * nnz].view(np.float64)
        return sp.csr_matrix((val.copy(), idx.copy(), ptr.copy()), shape=(nr, nc))

    def prolongation(self):
        return self._csr(self.export(2))

    def lor_conforming(self):
        return self._csr(self.export(3))

    def blocks(self):
        v = self.export(4).view(np.int64)
        nb = int(v[0])
        ptr = v[1:nb + 2]
        dofs = v[nb + 2:]
        return [dofs[ptr[i]:ptr[i + 1]].copy() for i in range(nb)]

    def block_inverses(self):
        """Inverses of the V_e blocks (FP64), in the order of blocks()."""
        v = self.export(8).view(np.float64)
        out, o = [], 0
        for b in self.blocks():
            k = len(b)
            out.append(v[o:o + k * k].reshape(k, k).copy())
            o += k * k
        return out

    def cg_coefficients(self):
        """alpha_k, beta_k of the last finished pcg_solve: two arrays of
        shape (rows, max_nrhs)."""
        v = self.export(9).view(np.float64)
        rows, hs = int(v[0]), int(v[1])
        a = v[2:2 + rows * hs].reshape(rows, hs).copy()
        b = v[2 + rows * hs:2 + 2 * rows * hs].reshape(rows, hs).copy()
        return a, b

    def node_coords(self):
        return self.export(5).view(np.float64).reshape(-1, self.mesh.dim)

    def amg_levels(self):
        v = self.export(6).view(np.int64)
        return v[1:1 + int(v[0])].tolist()

    def amg_level_stats(self):
        """(rows, nnz of A, nnz of P) per AMG level, finest first."""
        v = self.export(6).view(np.int64)
        n = int(v[0])
        return list(zip(*(v[1 + k * n:1 + (k + 1) * n].tolist() for k in range(3))))

    def summary(self):
        keys = ["ndof", "nconf", "nblocks", "max_block", "block_entries", "amg_levels", "nnz_AC", "nnz_P",
                "face_table_bytes", "device_bytes"]
        return dict(zip(keys, (int(v) for v in self.export(7).view(np.int64))))


class Batch:
    """hpdg_batch_*: continuous batching of single-RHS PCG solves, each on a
    stream of its own. Driven from one thread."""

    def __init__(self, max_active=8):
        h = C.c_void_p()
        _check(lib().hpdg_batch_create(int(max_active), C.byref(h)))
        self.h = h
        self.max_active = max_active
        # (operator, b, x) of every admitted solve until poll returns its tag:
        # the native batch holds raw pointers to them
        self._held = {}

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.hpdg_batch_destroy(self.h)   # synchronises; active solves stay unfinished
            self.h = None
        self._held = {}

    def admit(self, op: Operator, b, x, rtol=1e-8, maxit=1000, tag=0):
        """True if admitted, False when every slot is taken. The batch keeps
        op, b and x alive until poll() returns the solve's tag; tags of
        solves in flight must be distinct."""
        if int(tag) in self._held:
            raise ValueError(f"tag {tag} already has a solve in flight")
        code = lib().hpdg_batch_admit(self.h, op.h, _ptr(b, "b"), _ptr(x, "x"), float(rtol), int(maxit), int(tag))
        if code == -7:
            return False
        _check(code)
        self._held[int(tag)] = (op, b, x)
        return True

    def step(self, wait_us=0):
        """Advance; returns (active, retired-not-yet-polled)."""
        na, nd = C.c_int(), C.c_int()
        _check(lib().hpdg_batch_step(self.h, int(wait_us), C.byref(na), C.byref(nd)))
        return na.value, nd.value

    def poll(self, cap=64):
        """Retired solves: list of (tag, status, info dict)."""
        tags = (C.c_int64 * cap)()
        codes = (C.c_int * cap)()
        info = (SolveInfo * cap)()
        n = C.c_int()
        _check(lib().hpdg_batch_poll(self.h, cap, tags, codes, info, C.byref(n)))
        out = [(int(tags[i]), int(codes[i]), info[i].as_dict()) for i in range(n.value)]
        for t, _, _ in out:
            self._held.pop(t, None)
        return out
