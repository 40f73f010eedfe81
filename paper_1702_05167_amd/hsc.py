"""ctypes binding of libhsc (include/hsc.h, include/hsc_kernels.h).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  PyTorch provides device memory (tensors) and the HIP stream.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhsc.so")

HSC_DIAG_GR, HSC_DIAG_GL, HSC_TRANS, HSC_SPECTRAL_LR = 1, 2, 4, 8
HSC_BOND_GR, HSC_BOND_GL = 16, 32
STATUS = {0: "HSC_OK", -1: "HSC_E_ARG", -2: "HSC_E_NOT_SYMMETRIC", -3: "HSC_E_SINGULAR",
          -4: "HSC_E_NONFINITE", -5: "HSC_E_OOM", -6: "HSC_E_HIP", -7: "HSC_E_UNSTABLE"}


class HscError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Contact(C.Structure):
    _fields_ = [("n_sites", C.c_int64), ("sites", C.POINTER(C.c_int64)), ("lead_onsite", C.c_double),
                ("lead_hopping", C.c_double), ("coupling", C.c_double)]


class TreeOpts(C.Structure):
    _fields_ = [("coords", C.POINTER(C.c_int32)), ("split_mask", C.c_int32), ("leaf_side", C.c_int32),
                ("method", C.c_int32), ("dense_contacts", C.c_int32)]


class Outputs(C.Structure):
    _fields_ = [("diag_gr", C.c_void_p), ("diag_gl", C.c_void_p), ("trans", C.c_void_p), ("spectral_lr", C.c_void_p),
                ("status", C.c_void_p), ("guard", C.c_void_p), ("bond_gr", C.c_void_p), ("bond_gl", C.c_void_p)]


class TreeStats(C.Structure):
    _fields_ = [("n_sites", C.c_int64), ("n_clusters", C.c_int32), ("depth", C.c_int32),
                ("max_cluster", C.c_int32), ("max_front", C.c_int32), ("max_ancestors", C.c_int32),
                ("n_leaves", C.c_int32), ("flops_per_energy", C.c_double), ("bytes_per_energy", C.c_double)]


class SolveOpts(C.Structure):
    _fields_ = [("eta", C.c_double), ("kT", C.c_double), ("mu_L", C.c_double), ("mu_R", C.c_double),
                ("want", C.c_uint32), ("batch", C.c_int32), ("guard_tau", C.c_double),
                ("guard_rounds", C.c_int32), ("precision", C.c_int32), ("graph", C.c_int32),
                ("tune", C.c_int32), ("complex3m", C.c_int32), ("slices", C.c_int32),
                ("potential", C.c_void_p), ("streams", C.c_int32)]


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("u_left", C.c_double),
                ("u_right", C.c_double)]


class ScfOpts(C.Structure):
    _fields_ = [("coupling", C.c_double), ("n0", C.c_void_p), ("mixing", C.c_double), ("max_iter", C.c_int32),
                ("tol", C.c_double), ("history", C.c_int32)]


_lib = None


def lib():
    """Load libhsc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    L.hsc_version.restype = C.c_char_p
    L.hsc_last_error.restype = C.c_char_p
    L.hsc_ctx_last_error.restype = C.c_char_p
    L.hsc_ctx_last_error.argtypes = [vp]
    L.hsc_ctx_create.argtypes = [i32, vp, C.POINTER(vp)]
    L.hsc_ctx_destroy.argtypes = [vp]
    L.hsc_tree_build.argtypes = [i64, vp, vp, vp, i32, C.POINTER(Contact), C.POINTER(TreeOpts), C.POINTER(vp)]
    L.hsc_tree_merge.argtypes = [vp, i32, vp, C.POINTER(vp)]
    L.hsc_tree_concat.argtypes = [i32, vp, C.POINTER(vp)]
    L.hsc_tree_stats_get.argtypes = [vp, C.POINTER(TreeStats)]
    L.hsc_tree_export.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.hsc_tree_destroy.argtypes = [vp]
    L.hsc_solve.argtypes = [vp, vp, i32, vp, C.POINTER(SolveOpts), vp, vp, vp, vp, vp, vp]
    L.hsc_solve_ex.argtypes = [vp, vp, i32, vp, C.POINTER(SolveOpts), C.POINTER(Outputs)]
    L.hsc_tree_bonds.argtypes = [vp, vp, vp]
    L.hsc_tree_build_custom.argtypes = [i64, vp, vp, vp, i32, C.POINTER(Contact), i32, vp, vp, C.POINTER(vp)]
    L.hsc_solve_batch.argtypes = [vp, i32, vp, vp, vp, C.POINTER(SolveOpts), vp, vp, vp, vp, vp, vp]
    L.hsc_sync.argtypes = [vp]
    L.hsc_ctx_profile.argtypes = [vp, i32]
    L.hsc_ctx_profile_read.argtypes = [vp, vp, i32]
    L.hsc_ctx_profile_bytes.argtypes = [vp, vp, i32]
    L.hsc_ctx_profile_launches.argtypes = [vp, i64, vp, C.POINTER(i64)]
    L.hsc_kern_zgemm.argtypes = [vp, i32, i32, i32, i32, i32, dbl, dbl, vp, i32, vp, i32, i32, vp, i32, vp, i32]
    L.hsc_kern_zgemm_tile.argtypes = [vp, i32, i32, i32, i32, i32, i32, dbl, dbl, vp, i32, vp, i32, i32, vp, i32, vp,
                                      i32]
    L.hsc_kern_zgemm_dd.argtypes = [vp, i32, i32, i32, i32, i32, i32, i32, vp, i32, vp, i32, i32, vp, i32, vp, i32]
    L.hsc_kern_zgemm_dd_noalloc.argtypes = [vp, i32, i32, i32, i32, i32, i32, vp, i32, vp, i32, i32, vp, i32, vp,
                                            i32]
    L.hsc_kern_zinv_batched.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp]
    L.hsc_kern_zinv_dd.argtypes = [vp, i32, vp, i32, vp, i32, vp, i32]
    L.hsc_kern_mfma_probe.argtypes = [vp, vp]
    L.hsc_kern_mfma_rate.argtypes = [vp, C.POINTER(dbl)]
    L.hsc_totals.argtypes = [vp, i32, i64, vp, vp, vp, vp]
    L.hsc_poisson_solve.argtypes = [vp, C.POINTER(Grid), vp, vp]
    L.hsc_density.argtypes = [vp, i32, i64, vp, vp, vp]
    L.hsc_scf.argtypes = [vp, vp, C.POINTER(Grid), i32, vp, vp, C.POINTER(SolveOpts), C.POINTER(ScfOpts), vp, vp,
                          C.POINTER(i32), vp]
    L.hsc_mlp_create.argtypes = [vp, i32, vp, C.POINTER(vp)]
    L.hsc_mlp_destroy.argtypes = [vp]
    L.hsc_mlp_n_params.argtypes = [vp, C.POINTER(i64)]
    L.hsc_mlp_set_params.argtypes = [vp, vp, vp]
    L.hsc_mlp_get_params.argtypes = [vp, vp, vp]
    L.hsc_mlp_forward.argtypes = [vp, vp, i64, vp, vp]
    L.hsc_mlp_grads.argtypes = [vp, vp, i64, vp, vp, vp, vp]
    L.hsc_mlp_train.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp]
    for name in ("hsc_ctx_create", "hsc_ctx_destroy", "hsc_tree_build", "hsc_tree_merge", "hsc_tree_concat",
                 "hsc_tree_stats_get",
                 "hsc_tree_export", "hsc_tree_destroy", "hsc_solve", "hsc_solve_ex", "hsc_solve_batch", "hsc_sync",
                 "hsc_tree_bonds", "hsc_tree_build_custom",
                 "hsc_ctx_profile", "hsc_ctx_profile_read", "hsc_ctx_profile_bytes", "hsc_ctx_profile_launches",
                 "hsc_kern_zgemm", "hsc_kern_zgemm_tile", "hsc_kern_zgemm_dd", "hsc_kern_zgemm_dd_noalloc",
                 "hsc_kern_zinv_batched",
                 "hsc_kern_zinv_dd",
                 "hsc_kern_mfma_probe",
                 "hsc_kern_mfma_rate", "hsc_totals", "hsc_poisson_solve", "hsc_density", "hsc_scf",
                 "hsc_mlp_create", "hsc_mlp_destroy", "hsc_mlp_n_params", "hsc_mlp_set_params",
                 "hsc_mlp_get_params", "hsc_mlp_forward", "hsc_mlp_grads", "hsc_mlp_train"):
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


def check(code):
    if code != 0:
        raise HscError(code, lib().hsc_last_error().decode())


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _dptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


class Context:
    """A HIP device and stream (torch's current stream unless given)."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the solver runs only on the HIP device")
        self.device = device
        self.torch_device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.torch_device)
        self.stream = stream
        h = C.c_void_p()
        check(lib().hsc_ctx_create(device, C.c_void_p(stream.cuda_stream), C.byref(h)))
        self.h = h

    def sync(self):
        check(lib().hsc_sync(self.h))

    PROFILE_KINDS = ("assemble", "inv_panel", "inv_swap", "inv_unscramble", "gemm", "gather",
                     "assemble_n", "diag", "guard", "dd_assemble", "dd_inv_panel", "dd_inv_swap",
                     "dd_inv_unscramble", "dd_gemm", "inv_super", "oz_split", "oz_gemm", "dd_inv_super",
                     "face_half", "face_sigma", "bonds")

    def profile_bytes(self) -> dict:
        """Algorithmic bytes per launch kind since profiling was enabled (slice products only)."""
        k = len(self.PROFILE_KINDS)
        buf = np.zeros(k)
        check(lib().hsc_ctx_profile_bytes(self.h, _ptr(buf), k))
        return {name: float(buf[i]) for i, name in enumerate(self.PROFILE_KINDS)}

    def profile(self, enable: bool):
        check(lib().hsc_ctx_profile(self.h, 1 if enable else 0))

    def profile_read(self) -> dict:
        k = len(self.PROFILE_KINDS)
        buf = np.zeros(3 * k)
        check(lib().hsc_ctx_profile_read(self.h, _ptr(buf), k))
        return {name: dict(launches=buf[3 * i], ms=buf[3 * i + 1], flops=buf[3 * i + 2])
                for i, name in enumerate(self.PROFILE_KINDS)}

    PROFILE_PHASES = ("other", "inverse", "fold", "extract_g", "fold_n", "extract_p")

    def profile_launches(self) -> np.ndarray:
        """[(kind, flops, ms, phase)] of every timed launch since profile(True) (call after sync());
        phase indexes PROFILE_PHASES."""
        cnt = C.c_int64()
        check(lib().hsc_ctx_profile_launches(self.h, 0, None, C.byref(cnt)))
        buf = np.zeros(4 * max(int(cnt.value), 1))
        check(lib().hsc_ctx_profile_launches(self.h, cnt.value, _ptr(buf), C.byref(cnt)))
        return buf[:4 * int(cnt.value)].reshape(-1, 4)

    def close(self):
        if getattr(self, "h", None):
            lib().hsc_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Tree:
    """Nested-dissection cluster tree of one device (host object)."""

    def __init__(self, handle, n):
        self.h = handle
        self.n = n

    @classmethod
    def build(cls, n, indptr, indices, values, coords, contacts, split_mask=7, leaf_side=8, dense=False,
              graph=False):
        """contacts: [(sites, lead_onsite, lead_hopping, coupling)] for left, right.  dense=True:
        each contact is a whole end face with a lead continuing the face lattice (dense
        self-energy block); otherwise every contact site has its own 1D lead.  graph=True: nested
        dissection from the sparsity of H alone (coords unused, leaf_side = largest leaf in sites)."""
        indptr = np.ascontiguousarray(indptr, dtype=np.int64)
        indices = np.ascontiguousarray(indices, dtype=np.int32)
        vals = np.ascontiguousarray(np.asarray(values, dtype=np.complex128)).view(np.float64)
        coords = np.ascontiguousarray(np.zeros((n, 3)) if coords is None else coords, dtype=np.int32)
        keep = [indptr, indices, vals, coords]
        carr = (Contact * len(contacts))()
        for k, (sites, eps0, tl, tc) in enumerate(contacts):
            s = np.ascontiguousarray(sites, dtype=np.int64)
            keep.append(s)
            carr[k] = Contact(len(s), s.ctypes.data_as(C.POINTER(C.c_int64)), eps0, tl, tc)
        opts = TreeOpts(coords.ctypes.data_as(C.POINTER(C.c_int32)), split_mask, leaf_side, int(bool(graph)),
                        int(bool(dense)))
        h = C.c_void_p()
        check(lib().hsc_tree_build(n, _ptr(indptr), _ptr(indices), _ptr(vals), len(contacts), carr,
                                   C.byref(opts), C.byref(h)))
        return cls(h, n)

    @classmethod
    def from_device(cls, dev, leaf_side=8, transverse=False, dense=False, graph=False):
        """Tree of a synthetic device; transverse=True never cuts the transport axis (x), so every
        cluster spans the device from one contact to the other; dense=True: whole-face leads;
        graph=True: graph nested dissection (leaf_side = largest leaf in sites)."""
        mask = 0
        for a in dev.split_axes:
            if not (transverse and a == 0):
                mask |= 1 << a
        contacts = [(c.sites, c.lead_onsite, c.lead_hopping, c.coupling) for c in dev.contacts]
        return cls.build(dev.n, dev.indptr, dev.indices, dev.values, dev.coords, contacts, mask, leaf_side, dense,
                         graph)

    @classmethod
    def build_custom(cls, n, indptr, indices, values, contacts, cluster_of_site, parent):
        """Tree of the caller's partition: cluster_of_site [n], parent [n_clusters] (-1: the root)."""
        indptr = np.ascontiguousarray(indptr, dtype=np.int64)
        indices = np.ascontiguousarray(indices, dtype=np.int32)
        vals = np.ascontiguousarray(np.asarray(values, dtype=np.complex128)).view(np.float64)
        cos = np.ascontiguousarray(cluster_of_site, dtype=np.int32)
        par = np.ascontiguousarray(parent, dtype=np.int32)
        keep = [indptr, indices, vals, cos, par]
        carr = (Contact * len(contacts))()
        for k, (sites, eps0, tl, tc) in enumerate(contacts):
            s = np.ascontiguousarray(sites, dtype=np.int64)
            keep.append(s)
            carr[k] = Contact(len(s), s.ctypes.data_as(C.POINTER(C.c_int64)), eps0, tl, tc)
        h = C.c_void_p()
        check(lib().hsc_tree_build_custom(n, _ptr(indptr), _ptr(indices), _ptr(vals), len(contacts), carr,
                                          len(par), _ptr(cos), _ptr(par), C.byref(h)))
        return cls(h, n)

    @classmethod
    def slab_chain(cls, dev, axis=0):
        """The degenerate tree of Section 2.2: one cluster per plane along `axis`, each the child of
        the next (the root is the last plane), which makes the method the slab recursion of
        Section 2.1."""
        x = np.asarray(dev.coords)[:, axis].astype(np.int64)
        planes = np.unique(x)
        cos = np.searchsorted(planes, x)
        parent = np.arange(1, len(planes) + 1)
        parent[-1] = -1
        contacts = [(c.sites, c.lead_onsite, c.lead_hopping, c.coupling) for c in dev.contacts]
        return cls.build_custom(dev.n, dev.indptr, dev.indices, dev.values, contacts, cos, parent)

    def stats(self) -> dict:
        s = TreeStats()
        check(lib().hsc_tree_stats_get(self.h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in TreeStats._fields_}

    def export(self) -> dict:
        st = self.stats()
        nc = st["n_clusters"]
        perm = np.empty(self.n, np.int64)
        parent = np.empty(nc, np.int32)
        first = np.empty(nc, np.int32)
        size = np.empty(nc, np.int32)
        fptr = np.empty(nc + 1, np.int64)
        check(lib().hsc_tree_export(self.h, _ptr(perm), _ptr(parent), _ptr(first), _ptr(size), _ptr(fptr), None))
        fs = np.empty(max(1, int(fptr[-1])), np.int64)
        check(lib().hsc_tree_export(self.h, None, None, None, None, None, _ptr(fs)))
        return dict(perm=perm, parent=parent, first=first, size=size, front_ptr=fptr, front=fs[:fptr[-1]])

    def bonds(self) -> np.ndarray:
        """int64 [n_bonds, 2]: the pairs (i, j), i < j, with H_ij != 0, in the solver's bond order."""
        cnt = C.c_int64(0)
        check(lib().hsc_tree_bonds(self.h, None, C.byref(cnt)))
        out = np.empty((max(cnt.value, 1), 2), np.int64)
        check(lib().hsc_tree_bonds(self.h, _ptr(out), C.byref(cnt)))
        return out[:cnt.value]

    def merge(self, ids) -> "Tree":
        ids = np.ascontiguousarray(ids, dtype=np.int32)
        h = C.c_void_p()
        check(lib().hsc_tree_merge(self.h, len(ids), _ptr(ids), C.byref(h)))
        return Tree(h, self.n)

    @classmethod
    def concat(cls, trees) -> "Tree":
        """Forest of several devices, sites numbered device after device."""
        hs = (C.c_void_p * len(trees))(*[t.h.value for t in trees])
        h = C.c_void_p()
        check(lib().hsc_tree_concat(len(trees), hs, C.byref(h)))
        return cls(h, sum(t.n for t in trees))

    def close(self):
        if getattr(self, "h", None):
            lib().hsc_tree_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve(ctx: Context, tree: Tree, energies, eta=1e-8, kT=0.025, mu_L=0.1, mu_R=-0.1,
          want=HSC_DIAG_GR | HSC_DIAG_GL | HSC_TRANS, batch=0, out=None, sync=True, guard=False,
          guard_tau=0.0, guard_rounds=6, precision=3, graph=0, tune=0, complex3m=0, slices=0, potential=None,
          streams=0):
    """Solve all energies; returns a dict of device tensors (gr, gl, trans, spectral, status).
    slices: 8-bit slices per operand of the precision-3 products (0 = the library's 16, or 15).
    potential: device float64 [n] on-site potential energy added to H (site order), or None.
    streams: batches run round-robin on that many streams at once (each with its own plan), 0 or 1
    one after another."""
    import torch
    dev = ctx.torch_device
    e = torch.as_tensor(energies, dtype=torch.float64, device=dev).contiguous()
    ne, n = int(e.numel()), tree.n
    o = dict(out or {})
    if want & HSC_DIAG_GR and "gr" not in o:
        o["gr"] = torch.empty((ne, n), dtype=torch.complex128, device=dev)
    if want & HSC_DIAG_GL and "gl" not in o:
        o["gl"] = torch.empty((ne, n), dtype=torch.complex128, device=dev)
    if want & HSC_TRANS and "trans" not in o:
        o["trans"] = torch.empty(ne, dtype=torch.float64, device=dev)
    if want & HSC_SPECTRAL_LR and "spectral" not in o:
        o["spectral"] = torch.empty((ne, 2, n), dtype=torch.float64, device=dev)
    if "status" not in o:
        o["status"] = torch.empty(ne, dtype=torch.int32, device=dev)
    if guard and "guard" not in o:
        o["guard"] = torch.zeros((ne, tree.stats()["n_clusters"], 2), dtype=torch.float64, device=dev)
    if potential is not None:
        _check_vec(potential, n, "potential")
    opts = SolveOpts(eta, kT, mu_L, mu_R, want, batch, guard_tau, guard_rounds, precision, graph, tune, complex3m,
                     slices, _dptr(potential) if potential is not None else None, int(streams))
    if want & (HSC_BOND_GR | HSC_BOND_GL):
        nb = len(tree.bonds())
        for bit, key in ((HSC_BOND_GR, "bond_gr"), (HSC_BOND_GL, "bond_gl")):
            if want & bit and key not in o:
                o[key] = torch.empty((ne, nb), dtype=torch.complex128, device=dev)
        outs = Outputs(*[_dptr(o.get(k)) for k in ("gr", "gl", "trans", "spectral", "status", "guard", "bond_gr",
                                                  "bond_gl")])
        check(lib().hsc_solve_ex(ctx.h, tree.h, ne, _dptr(e), C.byref(opts), C.byref(outs)))
    else:
        check(lib().hsc_solve(ctx.h, tree.h, ne, _dptr(e), C.byref(opts), _dptr(o.get("gr")), _dptr(o.get("gl")),
                              _dptr(o.get("trans")), _dptr(o.get("spectral")), _dptr(o.get("status")),
                              _dptr(o.get("guard"))))
    if sync:
        ctx.sync()
    return o


def solve_batch(ctx: Context, trees, energies, eta=1e-8, kT=0.025, mu_L=0.1, mu_R=-0.1,
                want=HSC_DIAG_GR | HSC_DIAG_GL | HSC_TRANS, batch=0, outs=None, sync=True, precision=3, graph=0,
                tune=0, complex3m=0, slices=0, streams=0):
    """Several devices in one call (hsc_solve_batch); energies: one array for all devices or a
    list of per-device arrays.  Returns a list of output dicts (device tensors)."""
    import torch
    dev = ctx.torch_device
    nt = len(trees)
    if not isinstance(energies, (list, tuple)):
        energies = [energies] * nt
    es = []
    shared = None
    for e in energies:
        t = torch.as_tensor(e, dtype=torch.float64, device=dev).contiguous()
        if shared is not None and t.data_ptr() != shared.data_ptr() and torch.equal(t, shared):
            t = shared
        shared = shared if shared is not None else t
        es.append(t)
    outs = outs or [dict() for _ in range(nt)]
    for o, tr, e in zip(outs, trees, es):
        ne, n = int(e.numel()), tr.n
        if want & HSC_DIAG_GR and "gr" not in o:
            o["gr"] = torch.empty((ne, n), dtype=torch.complex128, device=dev)
        if want & HSC_DIAG_GL and "gl" not in o:
            o["gl"] = torch.empty((ne, n), dtype=torch.complex128, device=dev)
        if want & HSC_TRANS and "trans" not in o:
            o["trans"] = torch.empty(ne, dtype=torch.float64, device=dev)
        if want & HSC_SPECTRAL_LR and "spectral" not in o:
            o["spectral"] = torch.empty((ne, 2, n), dtype=torch.float64, device=dev)
        if "status" not in o:
            o["status"] = torch.empty(ne, dtype=torch.int32, device=dev)

    def arr(key):
        return (C.c_void_p * nt)(*[(o[key].data_ptr() if key in o else None) for o in outs])

    th = (C.c_void_p * nt)(*[t.h.value for t in trees])
    ne_arr = np.array([int(e.numel()) for e in es], np.int32)
    e_arr = (C.c_void_p * nt)(*[e.data_ptr() for e in es])
    opts = SolveOpts(eta, kT, mu_L, mu_R, want, batch, 0.0, 0, precision, graph, tune, complex3m, slices, None,
                     int(streams))
    check(lib().hsc_solve_batch(ctx.h, nt, th, _ptr(ne_arr), e_arr, C.byref(opts), arr("gr"), arr("gl"), arr("trans"),
                                arr("spectral"), arr("status"), None))
    if sync:
        ctx.sync()
    return outs


def _check_vec(t, n, name):
    import torch
    if not (isinstance(t, torch.Tensor) and t.dtype == torch.float64 and t.is_cuda and t.is_contiguous() and
            t.numel() == n):
        raise ValueError(f"{name} must be a contiguous float64 device tensor of {n} values")


def poisson_solve(ctx: Context, grid, rho, u_left=0.0, u_right=0.0, out=None):
    """hsc_poisson_solve: U on the (nx, ny, nz) grid for the source rho (device float64 [n]) with
    lead planes at u_left (x = -1) and u_right (x = nx)."""
    import torch
    n = int(grid[0]) * int(grid[1]) * int(grid[2])
    _check_vec(rho, n, "rho")
    u = torch.empty(n, dtype=torch.float64, device=rho.device) if out is None else out
    _check_vec(u, n, "out")
    g = Grid(int(grid[0]), int(grid[1]), int(grid[2]), float(u_left), float(u_right))
    check(lib().hsc_poisson_solve(ctx.h, C.byref(g), _dptr(rho), _dptr(u)))
    return u


def density(ctx: Context, weights, gl):
    """hsc_density: sum_e w_e Im G^<_ii / (2 pi) from diag G^< (device complex128 [n_e, n])."""
    import torch
    if not (isinstance(gl, torch.Tensor) and gl.dtype == torch.complex128 and gl.is_cuda and gl.dim() == 2):
        raise ValueError("gl must be a complex128 device tensor of shape [n_e, n]")
    ne, n = int(gl.shape[0]), int(gl.shape[1])
    _check_vec(weights, ne, "weights")
    d = torch.empty(n, dtype=torch.float64, device=gl.device)
    check(lib().hsc_density(ctx.h, ne, n, _dptr(weights), _dptr(gl.contiguous()), _dptr(d)))
    ctx.sync()
    return d


def scf(ctx: Context, tree: Tree, grid, energies, weights, u_left=0.0, u_right=0.0, coupling=0.0, n0=None,
        mixing=0.5, max_iter=10, tol=0.0, u0=None, eta=1e-8, kT=0.025, mu_L=0.1, mu_R=-0.1, batch=0,
        precision=3, tune=0, complex3m=0, slices=0, history=0):
    """hsc_scf: the self-consistent NEGF-Poisson loop; returns (u, density, residuals) with u and
    density device float64 [n] and residuals a numpy array (one per iteration run).  history > 0
    mixes by Anderson's method over that many past steps, 0 linearly."""
    import torch
    dev = ctx.torch_device
    n = tree.n
    e = torch.as_tensor(energies, dtype=torch.float64, device=dev).contiguous()
    w = torch.as_tensor(weights, dtype=torch.float64, device=dev).contiguous()
    u = (torch.zeros(n, dtype=torch.float64, device=dev) if u0 is None else
         torch.as_tensor(u0, dtype=torch.float64, device=dev).clone().contiguous())
    _check_vec(w, e.numel(), "weights")
    _check_vec(u, n, "u0")
    if n0 is not None:
        n0 = torch.as_tensor(n0, dtype=torch.float64, device=dev).contiguous()
        _check_vec(n0, n, "n0")
    dens = torch.empty(n, dtype=torch.float64, device=dev)
    g = Grid(int(grid[0]), int(grid[1]), int(grid[2]), float(u_left), float(u_right))
    opts = SolveOpts(eta, kT, mu_L, mu_R, HSC_DIAG_GL, batch, 0.0, 0, precision, 0, tune, complex3m, slices, None)
    so = ScfOpts(float(coupling), _dptr(n0) if n0 is not None else None, float(mixing), int(max_iter), float(tol),
                 int(history))
    its = C.c_int32(0)
    res = np.zeros(max(int(max_iter), 1))
    check(lib().hsc_scf(ctx.h, tree.h, C.byref(g), int(e.numel()), _dptr(e), _dptr(w), C.byref(opts), C.byref(so),
                        _dptr(u), _dptr(dens), C.byref(its), _ptr(res)))
    return u, dens, res[:its.value]


def totals(ctx: Context, out: dict, n: int):
    """Per-energy (DOS, electrons per unit energy, contact-injected DOS) from solve outputs:
    device float64 [n_e, 3]; columns whose input is absent stay zero."""
    import torch
    ref = next(out[k] for k in ("gr", "gl", "spectral") if k in out)
    ne = int(ref.shape[0])
    t = torch.zeros((ne, 3), dtype=torch.float64, device=ref.device)
    check(lib().hsc_totals(ctx.h, ne, n, _dptr(out.get("gr")), _dptr(out.get("gl")), _dptr(out.get("spectral")),
                           _dptr(t)))
    return t


# ---- kernel-level entry points -------------------------------------------------------------------

def kern_zgemm(ctx, opA, opB, alpha, A, B, beta=0, C_=None, D=None, tile=0):
    """D = alpha op(A) op(B) + beta C on device complex128 tensors (row-major 2D), tile shape `tile`."""
    import torch
    M = A.shape[0] if opA == 0 else A.shape[1]
    K = A.shape[1] if opA == 0 else A.shape[0]
    N = B.shape[1] if opB == 0 else B.shape[0]
    if D is None:
        D = torch.empty((M, N), dtype=torch.complex128, device=A.device)
    alpha = complex(alpha)
    check(lib().hsc_kern_zgemm_tile(ctx.h, tile, opA, opB, M, N, K, alpha.real, alpha.imag, _dptr(A), A.stride(0),
                               _dptr(B), B.stride(0), beta, _dptr(C_) if C_ is not None else None,
                               C_.stride(0) if C_ is not None else 0, _dptr(D), D.stride(0)))
    return D


def kern_zgemm_dd(ctx, opA, opB, A, B, negate=0, beta=0, C_=None, D=None, config=0):
    """D = (-1)^negate op(A) op(B) + beta C in complex double-double.  A, B, C, D: device float64
    tensors of shape (rows, cols, 4) holding (re hi, re lo, im hi, im lo) per element.  config 0-2:
    tiles of the FP64 vector-unit kernel; 3: 16 8-bit slices per operand on the integer matrix cores;
    4: 15 slices."""
    import torch
    M = A.shape[0] if opA == 0 else A.shape[1]
    K = A.shape[1] if opA == 0 else A.shape[0]
    N = B.shape[1] if opB == 0 else B.shape[0]
    if D is None:
        D = torch.empty((M, N, 4), dtype=torch.float64, device=A.device)
    for t in (A, B, D) + ((C_,) if C_ is not None else ()):
        if t.dim() != 3 or t.shape[2] != 4 or t.stride(2) != 1 or t.stride(1) != 4:
            raise ValueError("double-double operands are (rows, cols, 4) tensors with contiguous elements")
    check(lib().hsc_kern_zgemm_dd(ctx.h, config, opA, opB, M, N, K, negate, _dptr(A), A.stride(0) // 4,
                                  _dptr(B), B.stride(0) // 4, beta, _dptr(C_) if C_ is not None else None,
                                  C_.stride(0) // 4 if C_ is not None else 0, _dptr(D), D.stride(0) // 4))
    return D


def kern_zgemm_dd_noalloc(ctx, opA, opB, A, B, D, negate=0, beta=0, C_=None, sync=True):
    """hsc_kern_zgemm_dd_noalloc: the config-3 double-double product into the caller's D, with the
    library's static device scratch (no allocation, asynchronous; sync=True waits on the stream).
    Tensors as in kern_zgemm_dd."""
    M = A.shape[0] if opA == 0 else A.shape[1]
    K = A.shape[1] if opA == 0 else A.shape[0]
    N = B.shape[1] if opB == 0 else B.shape[0]
    for t in (A, B, D) + ((C_,) if C_ is not None else ()):
        if t.dim() != 3 or t.shape[2] != 4 or t.stride(2) != 1 or t.stride(1) != 4:
            raise ValueError("double-double operands are (rows, cols, 4) tensors with contiguous elements")
    if tuple(D.shape[:2]) != (M, N):
        raise ValueError("D must be (M, N, 4)")
    check(lib().hsc_kern_zgemm_dd_noalloc(ctx.h, opA, opB, M, N, K, negate, _dptr(A), A.stride(0) // 4, _dptr(B),
                                          B.stride(0) // 4, beta, _dptr(C_) if C_ is not None else None,
                                          C_.stride(0) // 4 if C_ is not None else 0, _dptr(D), D.stride(0) // 4))
    if sync:
        ctx.sync()
    return D


def kern_zinv_dd(ctx, X, matrix_cores=0):
    """Inverse of a square complex double-double matrix: X is a device float64 tensor (n, n, 4)
    (re hi, re lo, im hi, im lo), overwritten; returns (inverse, status).  matrix_cores=1: the
    super-panel updates on the integer matrix cores (as the precision-3 solve)."""
    import torch
    n = X.shape[0]
    if X.dim() != 3 or X.shape[1] != n or X.shape[2] != 4 or X.stride(2) != 1 or X.stride(1) != 4:
        raise ValueError("X must be a (n, n, 4) tensor with contiguous elements")
    Y = torch.empty_like(X)
    st = torch.empty(1, dtype=torch.int32, device=X.device)
    check(lib().hsc_kern_zinv_dd(ctx.h, n, _dptr(X), X.stride(0) // 4, _dptr(Y), Y.stride(0) // 4, _dptr(st),
                                 matrix_cores))
    return Y, st


def kern_zinv_batched(ctx, mats):
    """Invert a list of square device complex128 tensors (in place); returns (inverses, status)."""
    import torch
    cnt = len(mats)
    n = np.array([m.shape[0] for m in mats], np.int32)
    ld = np.array([m.stride(0) for m in mats], np.int32)
    outs = [torch.empty_like(m) for m in mats]
    ldy = np.array([o.stride(0) for o in outs], np.int32)
    X = (C.c_void_p * cnt)(*[m.data_ptr() for m in mats])
    Y = (C.c_void_p * cnt)(*[o.data_ptr() for o in outs])
    st = torch.empty(cnt, dtype=torch.int32, device=mats[0].device)
    check(lib().hsc_kern_zinv_batched(ctx.h, cnt, _ptr(n), X, _ptr(ld), Y, _ptr(ldy), _dptr(st)))
    return outs, st


def kern_mfma_probe(ctx):
    import torch
    out = torch.empty(256, dtype=torch.float64, device=ctx.torch_device)
    check(lib().hsc_kern_mfma_probe(ctx.h, _dptr(out)))
    return out


def kern_mfma_rate(ctx) -> float:
    """Achievable FP64 matrix-core rate of the device in TFLOP/s (an MFMA-only kernel, timed)."""
    r = C.c_double()
    check(lib().hsc_kern_mfma_rate(ctx.h, C.byref(r)))
    return float(r.value)
