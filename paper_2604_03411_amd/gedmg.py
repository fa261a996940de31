"""Python binding of the gedmg C ABI (include/gedmg.h).

Argument marshalling only: every step of the hot path runs in the HIP
library `libgedmg.so`.  Device arrays are torch tensors on the current HIP
device; the torch current stream is handed to the library.  Importing this
module without the built library raises immediately (there is no CPU
fallback).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgedmg.so")

FP64, BF16, FP16 = 0, 1, 2
PRECISIONS = {"fp64": FP64, "bf16": BF16, "fp16": FP16}

ERRORS = {
    -1: "GEDMG_E_ARG", -2: "GEDMG_E_SHAPE", -3: "GEDMG_E_NONFINITE", -4: "GEDMG_E_LOCAL_NOCONV",
    -5: "GEDMG_E_NEWTON_NOCONV", -6: "GEDMG_E_LINSOLVE", -7: "GEDMG_E_HIP", -8: "GEDMG_E_NOMEM",
    -9: "GEDMG_E_JNONPOS",
}


class GedmgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Mesh(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_nodes", C.c_int32), ("n_elems", C.c_int32),
                ("X", C.POINTER(C.c_double)), ("conn", C.POINTER(C.c_int32))]


class Material(C.Structure):
    _fields_ = [(n, C.c_double) for n in
                ("mu_e", "lambda_e", "eta_d", "kappa_d", "c_d", "beta_d", "gamma_d")]


class Icnn(C.Structure):
    _fields_ = [("n_in", C.c_int32), ("width", C.c_int32), ("n_hidden", C.c_int32),
                ("monotone_mask", C.c_int32), ("theta", C.POINTER(C.c_double))]


class Dirichlet(C.Structure):
    _fields_ = [("n", C.c_int32), ("dof", C.c_void_p), ("value", C.c_void_p)]


class SolverOpts(C.Structure):
    _fields_ = [("max_newton", C.c_int32), ("max_krylov", C.c_int32), ("max_local", C.c_int32),
                ("newton_rtol", C.c_double), ("newton_atol", C.c_double), ("krylov_rtol", C.c_double),
                ("krylov_forcing", C.c_int32), ("refine_max", C.c_int32), ("refine_rtol", C.c_double),
                ("scheme", C.c_int32), ("newton_rscale", C.c_double), ("krylov_method", C.c_int32)]

KRYLOV = {"cg": 0, "bicgstab": 1}

SCHEMES = {"monolithic": 0, "staggered": 1}


# Defaults of gedmg_solver_opts (include/gedmg.h); the bindings pass every field.
SOLVER_DEFAULTS = dict(max_newton=25, max_krylov=20000, max_local=100, newton_rtol=1e-10, newton_atol=0.0,
                       krylov_rtol=1e-12, krylov_forcing=True, refine_max=10, refine_rtol=1e-8,
                       scheme="monolithic", newton_rscale=1.0, krylov_method="cg")


def solver_opts(**kw):
    unknown = set(kw) - set(SOLVER_DEFAULTS)
    if unknown:
        raise GedmgError(-1, f"unknown solver options {sorted(unknown)}")
    o = dict(SOLVER_DEFAULTS, **kw)
    sch = o["scheme"]
    if isinstance(sch, str):
        if sch not in SCHEMES:
            raise GedmgError(-1, f"unknown scheme {sch!r}")
        sch = SCHEMES[sch]
    km = o["krylov_method"]
    if isinstance(km, str):
        if km not in KRYLOV:
            raise GedmgError(-1, f"unknown Krylov method {km!r}")
        km = KRYLOV[km]
    return SolverOpts(int(o["max_newton"]), int(o["max_krylov"]), int(o["max_local"]), float(o["newton_rtol"]),
                      float(o["newton_atol"]), float(o["krylov_rtol"]), 1 if o["krylov_forcing"] else 0,
                      int(o["refine_max"]), float(o["refine_rtol"]), int(sch), float(o["newton_rscale"]), int(km))


class NewtonReport(C.Structure):
    _fields_ = [("newton_iters", C.c_int32), ("krylov_iters_total", C.c_int32),
                ("n_yielded_qp", C.c_int32), ("status", C.c_int32),
                ("res_norm", C.c_double * 32), ("reaction", C.c_double), ("backtracks", C.c_int32),
                ("krylov_fallbacks", C.c_int32)]


class AdjointReport(C.Structure):
    _fields_ = [("n_checkpoints", C.c_int32), ("recomputed_steps", C.c_int32),
                ("newton_iters_total", C.c_int32), ("krylov_iters_total", C.c_int32),
                ("t_forward_s", C.c_double), ("t_recompute_s", C.c_double), ("t_reverse_s", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"gedmg HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        L.gedmg_last_error.restype = C.c_char_p
        L.gedmg_last_error.argtypes = [vp]
        L.gedmg_create.argtypes = [C.POINTER(vp), C.POINTER(Mesh), C.POINTER(Material),
                                   C.POINTER(Icnn), C.POINTER(Icnn), vp]
        L.gedmg_destroy.argtypes = [vp]
        L.gedmg_set_params.argtypes = [vp, C.POINTER(dp), C.POINTER(dp)]
        L.gedmg_csr.argtypes = [vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(vp), C.POINTER(vp)]
        L.gedmg_assemble.argtypes = [vp, vp, vp, vp, C.c_int, vp, vp, vp]
        if hasattr(L, "gedmg_assemble_static"):
            L.gedmg_assemble_static.argtypes = [vp, vp, vp, vp, C.c_int, vp, vp, vp]
        L.gedmg_status.argtypes = [vp]
        L.gedmg_energy_jet.argtypes = [vp, vp, i64, C.c_int, vp]
        L.gedmg_profile.argtypes = [vp, C.c_int]
        if hasattr(L, "gedmg_probe_mfma"):
            L.gedmg_probe_mfma.argtypes = [vp, i32, i32, vp]
        L.gedmg_profile_read.argtypes = [vp, C.POINTER(dp), C.POINTER(i32)]
        if hasattr(L, "gedmg_newton_step"):
            L.gedmg_newton_step.argtypes = [vp, C.POINTER(Dirichlet), C.POINTER(SolverOpts), C.c_int,
                                            vp, vp, vp, vp, vp, i32, C.POINTER(NewtonReport)]
        if hasattr(L, "gedmg_arclength_step"):
            L.gedmg_arclength_step.argtypes = [vp, C.POINTER(Dirichlet), C.POINTER(SolverOpts), dp, dp, dp,
                                               C.POINTER(dp), vp, vp, vp, vp, vp, i32, C.POINTER(NewtonReport)]
        if hasattr(L, "gedmg_adjoint"):
            L.gedmg_adjoint.argtypes = [vp, i32, C.POINTER(Dirichlet), vp, vp, i32, vp, i32,
                                        C.POINTER(SolverOpts), vp, vp, vp, C.POINTER(dp), C.POINTER(dp),
                                        C.POINTER(dp), C.POINTER(AdjointReport)]
        for name in ("gedmg_create", "gedmg_destroy", "gedmg_set_params", "gedmg_csr",
                     "gedmg_assemble", "gedmg_assemble_static", "gedmg_status", "gedmg_newton_step",
                     "gedmg_arclength_step", "gedmg_adjoint",
                     "gedmg_energy_jet", "gedmg_profile", "gedmg_profile_read", "gedmg_probe_mfma"):
            if hasattr(L, name):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


STATIC_MAX_QP = 262144  # GEDMG_STATIC_MAX_QP

EXPORTED = ("gedmg_last_error", "gedmg_create", "gedmg_destroy", "gedmg_set_params", "gedmg_csr",
            "gedmg_assemble", "gedmg_assemble_static", "gedmg_status", "gedmg_newton_step",
            "gedmg_arclength_step", "gedmg_adjoint",
            "gedmg_energy_jet", "gedmg_profile", "gedmg_profile_read", "gedmg_probe_mfma")


def probe_mfma(blocks, iters):
    """Launch the matrix-core calibration probe on the current stream; returns
    the number of FP64 16x16x4 products issued."""
    sink = torch.empty(blocks * 256, dtype=torch.float64, device="cuda")
    rc = lib().gedmg_probe_mfma(_dptr(sink), int(blocks), int(iters), _stream())
    if rc != 0:
        raise GedmgError(rc, "gedmg_probe_mfma failed")
    torch.cuda.synchronize()
    return blocks * 4 * 4 * iters


def _hip():
    return C.CDLL("libamdhip64.so")


def _dptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(None)


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _f64(t, dev):
    return torch.as_tensor(t, dtype=torch.float64, device=dev).contiguous()


def _check_array(t, numel, dev, name, dtype=torch.float64):
    """A caller's device array: contiguous, of the given dtype, size and device
    (checked here, before any launch, so that a wrong buffer cannot make a
    kernel index past its end)."""
    if not isinstance(t, torch.Tensor):
        raise GedmgError(-1, f"{name} must be a torch tensor")
    if t.dtype != dtype or not t.is_contiguous() or t.numel() != numel or t.device != dev:
        raise GedmgError(-1, f"{name} must be a contiguous {dtype} tensor of {numel} elements on {dev} "
                             f"(got {t.dtype}, {t.numel()} elements, contiguous={t.is_contiguous()}, {t.device})")
    return t


def _dof_index_array(idx, ndof, dev, name):
    """Host-checked int32 device array of dof indices in [0, ndof)."""
    a = np.asarray(idx.detach().cpu().numpy() if isinstance(idx, torch.Tensor) else idx).reshape(-1)
    if a.size and (not np.issubdtype(a.dtype, np.integer) or a.min() < 0 or a.max() >= ndof):
        raise GedmgError(-1, f"{name}: dof indices must be integers in [0, {ndof})")
    return torch.as_tensor(a.astype(np.int32), device=dev).contiguous()


class Context:
    """A gedmg context for one mesh, material and pair of networks."""

    def __init__(self, mesh, material: dict, energy_spec, theta_e, yield_spec, theta_y,
                 device="cuda"):
        dev = torch.device(device)
        if dev.type == "cuda" and dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.dev = dev
        self.dim = int(mesh.dim)
        self.n_nodes, self.n_elems = int(mesh.n_nodes), int(mesh.n_elems)
        self.nqp = 4 if self.dim == 2 else 8
        self.ndof = self.n_nodes * (self.dim + 1)
        self._X = np.ascontiguousarray(mesh.X, dtype=np.float64)
        self._conn = np.ascontiguousarray(mesh.conn, dtype=np.int32)
        self._te = np.ascontiguousarray(theta_e, dtype=np.float64)
        self._ty = np.ascontiguousarray(theta_y, dtype=np.float64)
        m = Mesh(self.dim, self.n_nodes, self.n_elems,
                 self._X.ctypes.data_as(C.POINTER(C.c_double)),
                 self._conn.ctypes.data_as(C.POINTER(C.c_int32)))
        mat = Material(*(float(material[k]) for k in
                         ("mu_e", "lambda_e", "eta_d", "kappa_d", "c_d", "beta_d", "gamma_d")))
        en = Icnn(energy_spec.n_in, energy_spec.width, energy_spec.n_hidden,
                  energy_spec.monotone_mask, self._te.ctypes.data_as(C.POINTER(C.c_double)))
        yl = Icnn(yield_spec.n_in, yield_spec.width, yield_spec.n_hidden,
                  yield_spec.monotone_mask, self._ty.ctypes.data_as(C.POINTER(C.c_double)))
        with torch.cuda.device(self.dev):
            h = C.c_void_p()
            rc = lib().gedmg_create(C.byref(h), C.byref(m), C.byref(mat), C.byref(en), C.byref(yl),
                                    _stream())
            self._h = h
            if rc != 0:
                msg = lib().gedmg_last_error(h).decode() if h.value else "create failed"
                if h.value:
                    lib().gedmg_destroy(h)
                self._h = None
                raise GedmgError(rc, msg)
        n_rows, nnz = C.c_int64(), C.c_int64()
        rp, cl = C.c_void_p(), C.c_void_p()
        self._check(lib().gedmg_csr(self._h, C.byref(n_rows), C.byref(nnz), C.byref(rp), C.byref(cl)))
        self.nnz = int(nnz.value)
        self._rowptr_ptr, self._col_ptr = rp.value, cl.value

    @classmethod
    def from_case(cls, case, device="cuda"):
        return cls(case.mesh, case.material, case.energy, case.theta_e, case.yield_, case.theta_y,
                   device)

    def _check(self, rc):
        if rc != 0:
            raise GedmgError(rc, lib().gedmg_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            lib().gedmg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- data
    def csr(self):
        """(rowptr, col) of the library's CSR pattern as int32 device tensors (copies)."""
        rp = torch.empty(self.ndof + 1, dtype=torch.int32, device=self.dev)
        cl = torch.empty(self.nnz, dtype=torch.int32, device=self.dev)
        torch.cuda.current_stream().synchronize()
        hip = _hip()
        hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
        for dst, src, n in ((rp, self._rowptr_ptr, rp.numel()), (cl, self._col_ptr, cl.numel())):
            rc = hip.hipMemcpy(C.c_void_p(dst.data_ptr()), C.c_void_p(src), n * 4, 3)
            if rc != 0:
                raise GedmgError(-7, f"hipMemcpy failed ({rc})")
        return rp, cl

    def set_params(self, theta_e=None, theta_y=None):
        te = None if theta_e is None else np.ascontiguousarray(theta_e, dtype=np.float64)
        ty = None if theta_y is None else np.ascontiguousarray(theta_y, dtype=np.float64)
        self._check(lib().gedmg_set_params(
            self._h, None if te is None else te.ctypes.data_as(C.POINTER(C.c_double)),
            None if ty is None else ty.ctypes.data_as(C.POINTER(C.c_double))))

    def fields(self, u, phi, kappa):
        return _f64(u, self.dev), _f64(phi, self.dev), _f64(kappa, self.dev)

    def _check_fields(self, u, phi, kappa):
        _check_array(u, self.dim * self.n_nodes, self.dev, "u")
        _check_array(phi, self.n_nodes, self.dev, "phi")
        _check_array(kappa, self.n_elems * self.nqp, self.dev, "kappa")

    def assemble(self, u, phi, kappa, precision="fp64", tangent=True, out=None, static_scratch=False):
        """Returns (R [ndof], K_vals [nnz] or None, kappa_trial [n_elems, nqp]) on the device.
        static_scratch: call gedmg_assemble_static (no allocation inside the
        library; pass `out` to allocate nothing on the Python side either)."""
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        if out is None:
            R = torch.empty(self.ndof, dtype=torch.float64, device=self.dev)
            K = torch.empty(self.nnz, dtype=torch.float64, device=self.dev) if tangent else None
            kt = torch.empty(self.n_elems, self.nqp, dtype=torch.float64, device=self.dev)
        else:
            R, K, kt = out
            _check_array(R, self.ndof, self.dev, "R")
            if K is not None:
                _check_array(K, self.nnz, self.dev, "K_vals")
                if K.data_ptr() % 16:
                    raise GedmgError(-1, "K_vals must be 16-byte aligned")
            _check_array(kt, self.n_elems * self.nqp, self.dev, "kappa_trial")
        self._check_fields(u, phi, kappa)
        fn = lib().gedmg_assemble_static if static_scratch else lib().gedmg_assemble
        self._check(fn(self._h, _dptr(u), _dptr(phi), _dptr(kappa), prec, _dptr(R), _dptr(K), _dptr(kt)))
        return R, K, kt

    def energy_jet(self, x, precision="fp64"):
        """Energy-network jet [n, 10] at inputs x [n, 3] (device tensors)."""
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        x = _f64(x, self.dev)
        if x.dim() != 2 or x.shape[1] != 3:
            raise GedmgError(-1, f"x must be [n, 3] network inputs (got shape {tuple(x.shape)})")
        n = x.shape[0]
        jet = torch.empty(n, 10, dtype=torch.float64, device=self.dev)
        self._check(lib().gedmg_energy_jet(self._h, _dptr(x), n, prec, _dptr(jet)))
        return jet

    def profile(self, enable=True):
        self._check(lib().gedmg_profile(self._h, 1 if enable else 0))

    def profile_read(self):
        """Summed ms of (inputs, jets, history, elements, fills) and the number of timed assemblies."""
        out = (C.c_double * 5)()
        n = C.c_int32()
        self._check(lib().gedmg_profile_read(self._h, out, C.byref(n)))
        return dict(inputs=out[0], jets=out[1], history=out[2], elements=out[3], fills=out[4],
                    calls=n.value)

    def newton_step(self, u, phi, kappa, bc_dofs, bc_vals, precision="fp64", reaction_dofs=None,
                    predictor_du=None, raise_on_error=True, **solver):
        """One load step in place on (u, phi, kappa): the predictor increment
        predictor_du ([dim][n_nodes], or None) is added to u, the prescribed dofs
        are set and Newton runs to convergence (gedmg_newton_step).  Solver
        options are the fields of gedmg_solver_opts as keywords.  Returns the
        report as a dict."""
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        self._check_fields(u, phi, kappa)
        dofs = _dof_index_array(bc_dofs, self.ndof, self.dev, "bc_dofs")
        vals = _f64(bc_vals, self.dev).reshape(-1)
        if vals.numel() != dofs.numel():
            raise GedmgError(-1, "bc_vals must hold one value per prescribed dof")
        bc = Dirichlet(int(dofs.numel()), C.c_void_p(dofs.data_ptr()), C.c_void_p(vals.data_ptr()))
        opts = solver_opts(**solver)
        pred = None
        if predictor_du is not None:
            pred = _check_array(_f64(predictor_du, self.dev), self.dim * self.n_nodes, self.dev, "predictor_du")
        rd = None
        nr = 0
        if reaction_dofs is not None:
            rd = _dof_index_array(reaction_dofs, self.ndof, self.dev, "reaction_dofs")
            nr = int(rd.numel())
        rep = NewtonReport()
        rc = lib().gedmg_newton_step(self._h, C.byref(bc), C.byref(opts), prec, _dptr(pred), _dptr(u), _dptr(phi),
                                     _dptr(kappa), _dptr(rd), nr, C.byref(rep))
        out = dict(status=rc, newton_iters=rep.newton_iters, krylov_iters=rep.krylov_iters_total,
                   n_yielded_qp=rep.n_yielded_qp, reaction=rep.reaction, backtracks=rep.backtracks,
                   krylov_fallbacks=rep.krylov_fallbacks,
                   res_norm=list(rep.res_norm[: min(rep.newton_iters + 1, 32)]))
        if rc != 0 and raise_on_error:
            self._check(rc)
        return out

    def arclength_step(self, u, phi, kappa, pattern_dofs, pattern_unit, lam, increment, ds, psi=1.0,
                       reaction_dofs=None, raise_on_error=True, phi_weight=1.0, **solver):
        """One arc-length increment in place on (u, phi, kappa) and the device
        array increment [ndof + 1] (gedmg_arclength_step; phi_weight weights
        the nonlocal damage dofs in the arc length).  Returns (lambda, report
        dict)."""
        self._check_fields(u, phi, kappa)
        _check_array(increment, self.ndof + 1, self.dev, "increment")
        dofs = _dof_index_array(pattern_dofs, self.ndof, self.dev, "pattern_dofs")
        vals = _f64(pattern_unit, self.dev).reshape(-1)
        if vals.numel() != dofs.numel() or dofs.numel() == 0:
            raise GedmgError(-1, "one unit value per prescribed dof, at least one dof")
        pat = Dirichlet(int(dofs.numel()), C.c_void_p(dofs.data_ptr()), C.c_void_p(vals.data_ptr()))
        opts = solver_opts(**solver)
        rd = None
        nr = 0
        if reaction_dofs is not None:
            rd = _dof_index_array(reaction_dofs, self.ndof, self.dev, "reaction_dofs")
            nr = int(rd.numel())
        lamc = C.c_double(float(lam))
        rep = NewtonReport()
        rc = lib().gedmg_arclength_step(self._h, C.byref(pat), C.byref(opts), float(ds), float(psi),
                                        float(phi_weight), C.byref(lamc),
                                        _dptr(increment), _dptr(u), _dptr(phi), _dptr(kappa), _dptr(rd), nr,
                                        C.byref(rep))
        out = dict(status=rc, newton_iters=rep.newton_iters, krylov_iters=rep.krylov_iters_total,
                   n_yielded_qp=rep.n_yielded_qp, reaction=rep.reaction, krylov_fallbacks=rep.krylov_fallbacks,
                   res_norm=list(rep.res_norm[: min(rep.newton_iters + 1, 32)]))
        if rc != 0 and raise_on_error:
            self._check(rc)
        return lamc.value, out

    def adjoint(self, path, checkpoint_every=5):
        """Loss and raw-parameter gradients of a load path (see LoadPath).

        Returns (loss, grad_energy, grad_yield, report dict); the path's
        initial state is left untouched (the solve runs on copies)."""
        n = path.n_steps
        dv = self.dev
        keep = []
        bcs = (Dirichlet * n)()
        for i, (bd, bv) in enumerate(path.bcs):
            d = _dof_index_array(bd, self.ndof, dv, f"bc_dofs of step {i + 1}")
            v = _f64(bv, dv).reshape(-1)
            if v.numel() != d.numel():
                raise GedmgError(-1, f"step {i + 1}: one value per prescribed dof")
            keep += [d, v]
            bcs[i] = Dirichlet(int(d.numel()), C.c_void_p(d.data_ptr()), C.c_void_p(v.data_ptr()))
        pred = None if path.predictor_du is None else _f64(path.predictor_du, dv)
        if pred is not None and pred.numel() != n * self.dim * self.n_nodes:
            raise GedmgError(-1, "predictor_du must hold n_steps x dim x n_nodes values")
        rd = _dof_index_array(path.reaction_dofs, self.ndof, dv, "reaction_dofs")
        tg = _f64(path.targets, dv)
        if tg.numel() != n:
            raise GedmgError(-1, "one target per load step")
        u, phi, kap = (_f64(t, dv).clone() for t in (path.u0, path.phi0, path.kappa0))
        self._check_fields(u, phi, kap)
        opts = solver_opts(**path.opts)
        ge = np.zeros(self._te.size)
        gy = np.zeros(self._ty.size)
        loss = C.c_double()
        rep = AdjointReport()
        self._check(lib().gedmg_adjoint(
            self._h, n, bcs, _dptr(pred), _dptr(rd), int(rd.numel()), _dptr(tg), int(checkpoint_every),
            C.byref(opts), _dptr(u), _dptr(phi), _dptr(kap), C.byref(loss),
            ge.ctypes.data_as(C.POINTER(C.c_double)), gy.ctypes.data_as(C.POINTER(C.c_double)),
            C.byref(rep)))
        report = {k: getattr(rep, k) for k, _ in AdjointReport._fields_}
        report["state"] = (u, phi, kap)
        return loss.value, ge, gy, report

    def status(self):
        rc = lib().gedmg_status(self._h)
        return rc

    def check_status(self):
        self._check(self.status())


class LoadPath:
    """A displacement-controlled load path: initial state, per-step Dirichlet
    sets (dofs, values), per-step predictor increments [n_steps][dim][n_nodes]
    (or None), reaction dofs, per-step reaction targets and solver options
    (keys of gedmg_solver_opts)."""

    def __init__(self, u0, phi0, kappa0, bcs, reaction_dofs, targets, predictor_du=None, **opts):
        self.u0, self.phi0, self.kappa0 = u0, phi0, kappa0
        self.bcs = list(bcs)
        self.n_steps = len(self.bcs)
        self.reaction_dofs = reaction_dofs
        self.targets = np.asarray(targets, dtype=np.float64)
        self.predictor_du = predictor_du
        self.opts = opts


class LoadPathLoss(torch.autograd.Function):
    """loss = sum_n (reaction_n - target_n)^2 over a load path as a function of
    the raw network parameters; the gradient comes from gedmg_adjoint, which
    computes it together with the loss in the forward call."""

    @staticmethod
    def forward(fctx, theta_e, theta_y, context, path, checkpoint_every=5):
        context.set_params(theta_e.detach().cpu().numpy(), theta_y.detach().cpu().numpy())
        loss, ge, gy, rep = context.adjoint(path, checkpoint_every)
        fctx.save_for_backward(torch.as_tensor(ge, dtype=theta_e.dtype, device=theta_e.device),
                               torch.as_tensor(gy, dtype=theta_y.dtype, device=theta_y.device))
        fctx.report = rep
        return torch.tensor(loss, dtype=theta_e.dtype, device=theta_e.device)

    @staticmethod
    def backward(fctx, g):
        ge, gy = fctx.saved_tensors
        return g * ge, g * gy, None, None, None


def load_path_loss(context, theta_e, theta_y, path, checkpoint_every=5):
    return LoadPathLoss.apply(theta_e, theta_y, context, path, checkpoint_every)
