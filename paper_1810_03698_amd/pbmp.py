"""ctypes binding of libpbmp.so (include/pbmp.h).

Argument marshalling only: every step of the method runs in the HIP
library.  Inputs may be numpy arrays (host) or torch tensors on the HIP
device (passed by device pointer); all are float64 except triangle indices
and groups (int32).  There is no CPU fallback: if the library is missing or
fails to load, ``load()`` raises.
"""

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpbmp.so")

HOST, DEVICE = 0, 1
MODE = {"direct": 0, "treecode": 1, "auto": 2}
PRECISION = {"fp64": 0, "mixed": 1}
STATUS = {0: "ok", -1: "bad argument", -2: "bad mesh", -3: "site outside",
          -4: "HIP error", -5: "out of device memory", -6: "call out of order",
          1: "GMRES not converged", 2: "SCF not converged"}


class Options(ctypes.Structure):
    _fields_ = [("eps_in", ctypes.c_double), ("eps_out", ctypes.c_double),
                ("kappa", ctypes.c_double), ("gauss_far", ctypes.c_int),
                ("near_eta", ctypes.c_double), ("mode", ctypes.c_int),
                ("theta", ctypes.c_double), ("order_P", ctypes.c_int),
                ("leaf_panels", ctypes.c_int), ("gmres_restart", ctypes.c_int),
                ("gmres_tol", ctypes.c_double), ("gmres_maxit", ctypes.c_int),
                ("scf_tol_debye", ctypes.c_double), ("scf_omega", ctypes.c_double),
                ("scf_maxit", ctypes.c_int), ("thole_a", ctypes.c_double),
                ("precision", ctypes.c_int), ("hip_stream", ctypes.c_void_p),
                ("warm_start", ctypes.c_int), ("verbose", ctypes.c_int)]


class Result(ctypes.Structure):
    _fields_ = [("where", ctypes.c_int),
                ("phi", ctypes.c_void_p), ("dphidn", ctypes.c_void_p),
                ("mu_diss", ctypes.c_void_p), ("mu_vac", ctypes.c_void_p),
                ("dG_kcal", ctypes.c_double), ("dG_solv_kcal", ctypes.c_double),
                ("dG_pol_kcal", ctypes.c_double),
                ("scf_iters", ctypes.c_int), ("scf_iters_vac", ctypes.c_int),
                ("gmres_iters_total", ctypes.c_int), ("matvecs", ctypes.c_int),
                ("final_relres", ctypes.c_double), ("t_setup_ms", ctypes.c_double),
                ("t_solve_ms", ctypes.c_double), ("t_matvec_ms", ctypes.c_double),
                ("G_vac_kcal", ctypes.c_double),
                ("dipole_vac_debye", ctypes.c_double * 3),
                ("dipole_diss_debye", ctypes.c_double * 3)]


class KernelStats(ctypes.Structure):
    _fields_ = [("p2p_ms", ctypes.c_double), ("m2p_ms", ctypes.c_double),
                ("p2m_ms", ctypes.c_double), ("matvec_ms", ctypes.c_double),
                ("p2p_launches", ctypes.c_int64), ("m2p_launches", ctypes.c_int64),
                ("matvec_calls", ctypes.c_int64), ("p2p_pairs", ctypes.c_double),
                ("m2p_pairs", ctypes.c_double)]


_lib = None

SYMBOLS = ["pbmp_default_options", "pbmp_create", "pbmp_set_mesh",
           "pbmp_set_sites", "pbmp_solve", "pbmp_matvec", "pbmp_rhs",
           "pbmp_site_fields", "pbmp_backward", "pbmp_last_error",
           "pbmp_destroy", "pbmp_kernel_stats", "pbmp_tree_export", "pbmp_set_stern",
           "pbmp_set_options", "pbmp_site_fields_noalloc", "pbmp_binding_energies",
           "pbmp_ligand_translation_gradient"]


def _torch_runtime_first():
    """torch ships its own copy of the HIP runtime.  Two runtimes share the
    device in one process only if torch's is initialised first (the other
    order leaves torch without a device), so initialise it before this
    library's when torch is present and sees a GPU."""
    try:
        import torch
    except ImportError:
        return
    if torch.cuda.is_available():
        torch.cuda.init()


def load():
    """Load libpbmp.so and declare its signatures.  Raises when missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libpbmp.so is not built (run __graft_entry__.build())")
    _torch_runtime_first()
    lib = ctypes.CDLL(LIB_PATH)
    P, D, I, L = ctypes.c_void_p, ctypes.c_double, ctypes.c_int, ctypes.c_int64
    lib.pbmp_default_options.argtypes = [ctypes.POINTER(Options)]
    lib.pbmp_default_options.restype = None
    lib.pbmp_create.argtypes = [ctypes.POINTER(Options), ctypes.POINTER(P)]
    lib.pbmp_set_mesh.argtypes = [P, L, P, L, P, I]
    lib.pbmp_set_sites.argtypes = [P, L, P, P, P, P, P, P, I]
    lib.pbmp_solve.argtypes = [P, ctypes.POINTER(Result)]
    lib.pbmp_matvec.argtypes = [P, P, P, I, I]
    lib.pbmp_rhs.argtypes = [P, P, P, I]
    lib.pbmp_site_fields.argtypes = [P, P, P, I]
    lib.pbmp_site_fields_noalloc.argtypes = [P, P, P]
    lib.pbmp_binding_energies.argtypes = [P, P, P, P]
    lib.pbmp_ligand_translation_gradient.argtypes = [P, L, P, P, P, I]
    lib.pbmp_backward.argtypes = [P, D, P, P, P, P, P, I]
    lib.pbmp_last_error.argtypes = [P]
    lib.pbmp_last_error.restype = ctypes.c_char_p
    lib.pbmp_destroy.argtypes = [P]
    lib.pbmp_destroy.restype = None
    lib.pbmp_kernel_stats.argtypes = [P, I, ctypes.POINTER(KernelStats)]
    lib.pbmp_tree_export.argtypes = [P] * 12
    lib.pbmp_set_stern.argtypes = [P, L, P, L, P, D, I]
    lib.pbmp_set_options.argtypes = [P, ctypes.POINTER(Options)]
    for name in ("pbmp_create", "pbmp_set_mesh", "pbmp_set_sites", "pbmp_solve",
                 "pbmp_matvec", "pbmp_rhs", "pbmp_site_fields", "pbmp_backward",
                 "pbmp_kernel_stats", "pbmp_tree_export", "pbmp_set_stern",
                 "pbmp_set_options", "pbmp_site_fields_noalloc", "pbmp_binding_energies",
                 "pbmp_ligand_translation_gradient"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


class PbmpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("pbmp error %d (%s): %s" % (code, STATUS.get(code, "?"), msg))
        self.code = code


def _is_torch(a):
    return type(a).__module__.startswith("torch")


class _Arg:
    """Pointer + address space for one argument; keeps host copies alive."""

    def __init__(self, a, dtype, count=None):
        self.keep = None
        if a is None:
            self.ptr, self.where = None, None
            return
        if _is_torch(a):
            import torch
            want = torch.float64 if dtype == np.float64 else torch.int32
            if a.dtype != want:
                raise TypeError("expected %s tensor" % want)
            if not a.is_contiguous():
                raise ValueError("tensor must be contiguous")
            if count is not None and a.numel() != count:
                raise ValueError("expected %d elements, got %d" % (count, a.numel()))
            self.keep = a
            self.ptr = a.data_ptr()
            self.where = DEVICE if a.is_cuda else HOST
        else:
            arr = np.ascontiguousarray(a, dtype=dtype)
            if count is not None and arr.size != count:
                raise ValueError("expected %d elements, got %d" % (count, arr.size))
            self.keep = arr
            self.ptr = arr.ctypes.data
            self.where = HOST


def _common_where(args):
    ws = {a.where for a in args if a.where is not None}
    if len(ws) > 1:
        raise ValueError("mixing host and device arguments in one call")
    return ws.pop() if ws else HOST


class Solver:
    """One library context: a mesh, sites and the solver options."""

    def __init__(self, eps_in=1.0, eps_out=80.0, kappa=0.125, gauss_far=3,
                 near_eta=2.0, mode="auto", theta=0.5, order_P=4,
                 leaf_panels=300, gmres_restart=50, gmres_tol=1e-6,
                 gmres_maxit=1000, scf_tol_debye=1e-6, scf_omega=0.7,
                 scf_maxit=200, thole_a=0.39, precision="mixed", stream=None,
                 warm_start=False, verbose=False):
        self.lib = load()
        o = Options()
        self.lib.pbmp_default_options(ctypes.byref(o))
        o.eps_in, o.eps_out, o.kappa = eps_in, eps_out, kappa
        o.gauss_far, o.near_eta = gauss_far, near_eta
        o.mode = MODE[mode] if isinstance(mode, str) else int(mode)
        o.theta, o.order_P, o.leaf_panels = theta, order_P, leaf_panels
        o.gmres_restart, o.gmres_tol, o.gmres_maxit = gmres_restart, gmres_tol, gmres_maxit
        o.scf_tol_debye, o.scf_omega, o.scf_maxit = scf_tol_debye, scf_omega, scf_maxit
        o.thole_a = thole_a
        o.precision = PRECISION[precision] if isinstance(precision, str) else int(precision)
        o.hip_stream = stream
        o.warm_start = int(bool(warm_start))
        o.verbose = int(bool(verbose))
        self.opts = o
        ctx = ctypes.c_void_p()
        rc = self.lib.pbmp_create(ctypes.byref(o), ctypes.byref(ctx))
        if rc != 0:
            raise PbmpError(rc, self.lib.pbmp_last_error(None).decode())
        self.ctx = ctx
        self.nt = self.nv = self.m = 0
        # advanced by every call that replaces the state a backward
        # differentiates (mesh, sites, Stern layer, solve), so that a caller
        # holding an earlier solve's number can tell that it is gone
        self.state_id = 0

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.pbmp_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, allow_warn=False):
        if rc < 0 or (rc > 0 and not allow_warn):
            raise PbmpError(rc, self.lib.pbmp_last_error(self.ctx).decode())
        return rc

    def set_mesh(self, verts, tris):
        nv = len(verts)
        nt = len(tris)
        v, t = _Arg(verts, np.float64, 3 * nv), _Arg(tris, np.int32, 3 * nt)
        self.state_id += 1
        self._check(self.lib.pbmp_set_mesh(self.ctx, nv, v.ptr, nt, t.ptr,
                                           _common_where([v, t])))
        self.nt, self.nv, self.nt2 = nt, nv, 0

    def set_options(self, **kw):
        """Change solver settings between solves (gmres_restart, gmres_tol,
        gmres_maxit, scf_tol_debye, scf_omega, scf_maxit, warm_start,
        verbose, precision)."""
        o = self.opts
        for k, v in kw.items():
            if k not in ("gmres_restart", "gmres_tol", "gmres_maxit", "scf_tol_debye",
                         "scf_omega", "scf_maxit", "warm_start", "verbose",
                         "precision"):
                raise ValueError("%s is fixed at creation" % k)
            if k == "precision":
                v = PRECISION[v] if isinstance(v, str) else int(v)
            setattr(o, k, int(v) if k in ("gmres_restart", "gmres_maxit", "scf_maxit",
                                          "warm_start", "verbose", "precision") else float(v))
        self._check(self.lib.pbmp_set_options(self.ctx, ctypes.byref(o)))

    def set_stern(self, verts, tris, eps_stern):
        """Enclosing ion-exclusion surface (see pbmp_set_stern); tris=None
        removes it."""
        self.state_id += 1
        if tris is None:
            self._check(self.lib.pbmp_set_stern(self.ctx, 0, None, 0, None, float(eps_stern), HOST))
            self.nt2 = 0
            return
        nv, nt = len(verts), len(tris)
        v, t = _Arg(verts, np.float64, 3 * nv), _Arg(tris, np.int32, 3 * nt)
        self._check(self.lib.pbmp_set_stern(self.ctx, nv, v.ptr, nt, t.ptr, float(eps_stern),
                                            _common_where([v, t])))
        self.nt2 = nt

    def set_sites(self, xyz, q, d, Q9, alpha, group=None):
        m = len(q)
        args = [_Arg(xyz, np.float64, 3 * m), _Arg(q, np.float64, m),
                _Arg(d, np.float64, 3 * m), _Arg(Q9, np.float64, 9 * m),
                _Arg(alpha, np.float64, m),
                _Arg(group, np.int32, m) if group is not None else _Arg(None, None)]
        w = _common_where(args)
        self.state_id += 1
        self._check(self.lib.pbmp_set_sites(self.ctx, m, *[a.ptr for a in args], w))
        self.m = m

    def solve(self, outputs=True):
        """Returns a dict with dG (kcal/mol), its two parts, counters and
        (if outputs) phi, dphidn [nt] and mu_diss, mu_vac [m,3] as numpy."""
        r = Result()
        r.where = HOST
        keep = {}
        if outputs:
            keep = dict(phi=np.empty(self.nt), dphidn=np.empty(self.nt),
                        mu_diss=np.empty((self.m, 3)), mu_vac=np.empty((self.m, 3)))
            r.phi, r.dphidn = keep["phi"].ctypes.data, keep["dphidn"].ctypes.data
            r.mu_diss, r.mu_vac = keep["mu_diss"].ctypes.data, keep["mu_vac"].ctypes.data
        self.state_id += 1
        rc = self._check(self.lib.pbmp_solve(self.ctx, ctypes.byref(r)), allow_warn=True)
        out = dict(status=rc, dG=r.dG_kcal, dG_solv=r.dG_solv_kcal,
                   dG_pol=r.dG_pol_kcal, G_vac=r.G_vac_kcal, scf_iters=r.scf_iters,
                   scf_iters_vac=r.scf_iters_vac, gmres_iters=r.gmres_iters_total,
                   matvecs=r.matvecs, relres=r.final_relres,
                   t_setup_ms=r.t_setup_ms, t_solve_ms=r.t_solve_ms,
                   t_matvec_ms=r.t_matvec_ms,
                   dipole_vac=np.array(r.dipole_vac_debye[:]),
                   dipole_diss=np.array(r.dipole_diss_debye[:]))
        out.update(keep)
        return out

    def matvec(self, x, transpose=False, out=None):
        n = 2 * self.nt + 2 * getattr(self, "nt2", 0)
        a = _Arg(x, np.float64, n)
        if out is None:
            out = np.empty(n) if a.where == HOST else _empty_like_torch(x)
        o = _Arg(out, np.float64, n)
        self._check(self.lib.pbmp_matvec(self.ctx, a.ptr, o.ptr, int(transpose),
                                         _common_where([a, o])))
        return out

    def rhs(self, p_total):
        a = _Arg(p_total, np.float64, 3 * self.m)
        out = np.empty(self.nt)
        if a.where == DEVICE:
            out = _empty_like_torch(p_total, self.nt)
        o = _Arg(out, np.float64, self.nt)
        self._check(self.lib.pbmp_rhs(self.ctx, a.ptr, o.ptr, _common_where([a, o])))
        return out

    def site_fields(self, x):
        a = _Arg(x, np.float64, 2 * self.nt)
        out = np.empty((self.m, 10))
        if a.where == DEVICE:
            out = _empty_like_torch(x, 10 * self.m).reshape(self.m, 10)
        o = _Arg(out, np.float64, 10 * self.m)
        self._check(self.lib.pbmp_site_fields(self.ctx, a.ptr, o.ptr,
                                              _common_where([a, o])))
        return out

    def site_fields_noalloc(self, x, out):
        """pbmp_site_fields_noalloc: x [2 nt] and out [m, 10] are float64
        torch tensors on the device; the library allocates nothing."""
        a = _Arg(x, np.float64, 2 * self.nt)
        o = _Arg(out, np.float64, 10 * self.m)
        if a.where != DEVICE or o.where != DEVICE:
            raise ValueError("site_fields_noalloc takes device tensors")
        self._check(self.lib.pbmp_site_fields_noalloc(self.ctx, a.ptr, o.ptr))
        return out

    def backward(self, dG_bar=1.0, verts=True, device=None):
        """Gradients of dG_bar * dG (see pbmp_backward).  Host numpy arrays by
        default; torch tensors on `device` when given (written by the library
        directly into device memory)."""
        shapes = dict(xyz=(self.m, 3), q=(self.m,), d=(self.m, 3), Q9=(self.m, 9))
        if verts:
            shapes["verts"] = (self.nv, 3)
        if device is None:
            g = {k: np.empty(v) for k, v in shapes.items()}
            ptr = lambda k: g[k].ctypes.data if k in g else None
            where = HOST
        else:
            import torch
            g = {k: torch.empty(v, dtype=torch.float64, device=device)
                 for k, v in shapes.items()}
            ptr = lambda k: g[k].data_ptr() if k in g else None
            where = DEVICE
        rc = self._check(self.lib.pbmp_backward(self.ctx, float(dG_bar), ptr("xyz"),
                                                ptr("q"), ptr("d"), ptr("Q9"),
                                                ptr("verts"), where), allow_warn=True)
        g["status"] = rc
        return g

    def ligand_translation_gradient(self, first_ligand_site, radii):
        """pbmp_ligand_translation_gradient: (g_t [3], number of ligand
        vertices, status)."""
        r = _Arg(radii, np.float64, self.m)
        g = np.empty(3)
        nlv = np.zeros(1, dtype=np.int64)
        rc = self._check(self.lib.pbmp_ligand_translation_gradient(
            self.ctx, int(first_ligand_site), r.ptr, g.ctypes.data, nlv.ctypes.data,
            _common_where([r])), allow_warn=True)
        return g, int(nlv[0]), rc

    def kernel_stats(self, enable=None):
        """Device time per kernel class (HIP events).  enable=1 starts
        collection (and resets), 0 stops, None just reads."""
        st = KernelStats()
        mode = -1 if enable is None else int(bool(enable))
        self._check(self.lib.pbmp_kernel_stats(self.ctx, mode, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in KernelStats._fields_}

    def tree(self):
        """The treecode octree and interaction lists of the current mesh
        (numpy arrays; see pbmp_tree_export)."""
        counts = np.zeros(4, dtype=np.int64)
        self._check(self.lib.pbmp_tree_export(self.ctx, counts.ctypes.data, *([None] * 10)))
        nbox, nleaf, nm, npp = (int(v) for v in counts)
        out = dict(perm=np.empty(self.nt, np.int32), box_range=np.empty(2 * nbox, np.int32),
                   box_level=np.empty(nbox, np.int32), box_centre=np.empty(3 * nbox),
                   box_radius=np.empty(2 * nbox), leaf_box=np.empty(nleaf, np.int32),
                   m2p_ptr=np.empty(nleaf + 1, np.int32), m2p_box=np.empty(max(nm, 1), np.int32),
                   p2p_ptr=np.empty(nleaf + 1, np.int32), p2p_box=np.empty(max(npp, 1), np.int32))
        order = ("perm", "box_range", "box_level", "box_centre", "box_radius", "leaf_box",
                 "m2p_ptr", "m2p_box", "p2p_ptr", "p2p_box")
        self._check(self.lib.pbmp_tree_export(self.ctx, counts.ctypes.data,
                                              *[out[k].ctypes.data for k in order]))
        out["box_range"] = out["box_range"].reshape(nbox, 2)
        out["box_centre"] = out["box_centre"].reshape(nbox, 3)
        out["box_radius"] = out["box_radius"].reshape(nbox, 2)
        out["m2p_box"] = out["m2p_box"][:nm]
        out["p2p_box"] = out["p2p_box"][:npp]
        return out


def binding_energies(complex_solver, receptor_solver, ligand_solver):
    """pbmp_binding_energies of three solved contexts: (ddG, dG_bind_vac,
    dG_bind_diss) in kcal/mol."""
    out = np.empty(3)
    lib = complex_solver.lib
    rc = lib.pbmp_binding_energies(complex_solver.ctx, receptor_solver.ctx, ligand_solver.ctx,
                                   out.ctypes.data)
    if rc != 0:
        raise PbmpError(rc, lib.pbmp_last_error(complex_solver.ctx).decode())
    return tuple(out)


def _empty_like_torch(t, n=None):
    import torch
    return torch.empty(n if n is not None else t.numel(), dtype=torch.float64,
                       device=t.device)
