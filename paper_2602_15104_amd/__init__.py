"""Python binding of libcmbhip (FP64 CMB Boltzmann hot path on MI355X).

Argument marshalling only: every step of the path runs in the C++ host table
builder and the HIP kernels of ``libcmbhip.so``.  PyTorch provides device
memory and the current HIP stream.  The library is loaded from this folder;
if it is missing the import fails loudly (build it with
``python -m paper_2602_15104_amd.build``).

Names follow include/cmbhip.h:
    defaults(), build_tables(), Tables.export(), Context,
    Context.perturb(), Context.los(), Context.cl(), Context.solve(),
and the convenience ``solve_batch`` that allocates torch outputs.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("CMBHIP_LIBRARY") or os.path.join(_HERE, "libcmbhip.so")


class _MissingLibrary:
    """Stands in for the library until it is built (or rebuilt, when the file
    on disk lacks a symbol of this binding); every use raises."""

    def __init__(self, why: str = "not found"):
        self.why = why

    def __getattr__(self, name):
        raise RuntimeError(f"libcmbhip.so {self.why} at {LIB_PATH}: build it with "
                           f"`python -m paper_2602_15104_amd.build` (no CPU fallback exists)")

CMB_OK = 0
ERRORS = {1: "CMB_E_INVALID", 2: "CMB_E_CONFLICT", 3: "CMB_E_NEG_NMASSLESS", 4: "CMB_E_ROOT", 5: "CMB_E_DEVICE",
          6: "CMB_E_NOMEM", 7: "CMB_E_UNSUPPORTED"}
MODE_STATUS = {0: "OK", 1: "MAX_STEPS", 2: "NONFINITE", 3: "STEP_UNDERFLOW"}

# exported symbols (kept in step with include/cmbhip.h; a CPU test checks this)
EXPORTS = ["cmb_abi_version", "cmb_defaults", "cmb_last_error", "cmb_tables_build", "cmb_tables_destroy",
           "cmb_tables_export", "cmb_ctx_create", "cmb_ctx_destroy", "cmb_solve_workspace_bytes", "cmb_perturb",
           "cmb_los", "cmb_cl", "cmb_solve", "cmb_perturb_pk", "cmb_transfer_kgrid", "cmb_spectra_on_grid",
           "cmb_bessel3_table", "cmb_los_bessel3", "cmb_perturb_matter", "cmb_lensing_potential",
           "cmb_lensed_cl", "cmb_perturb_record", "cmb_perturb_replay", "cmb_perturb_checkpoint",
           "cmb_perturb_segment", "cmb_jacobian", "cmb_gradient",
           "cmb_spectra_adjoint", "cmb_state_rows", "cmb_sources_adjoint",
           "cmb_server_create", "cmb_server_submit", "cmb_server_wait",
           "cmb_server_destroy", "cmb_server_selftest_arena", "cmb_solve_noalloc", "cmb_noalloc_scratch_bytes"]


class CmbError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = _lib.cmb_last_error().decode()
        super().__init__(f"{where}: {ERRORS.get(code, code)}: {msg}")
        self.code = code
        self.name = ERRORS.get(code, str(code))


class CCosmo(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in (
        "h", "omega_b", "omega_cdm", "A_s", "n_s", "tau_reio", "z_reio", "Delta_z_reio", "z_reio_He",
        "Delta_z_reio_He", "exp_reio", "YHe", "TCMB0", "Neff", "N_nu_massless", "T_nu_massless", "N_nu_massive",
        "m_nu_massive", "T_nu_massive")]


class CPrec(ctypes.Structure):
    _fields_ = ([(n, ctypes.c_int) for n in ("ell_gamma", "ell_pol", "ell_nu", "n_q", "ell_ncdm", "max_steps",
                                             "n_tab")] +
                [(n, ctypes.c_double) for n in ("rtol_small", "rtol_large", "atol_small", "atol_large", "k_split",
                                                "R_tc", "R_large", "k_pivot", "pcoeff", "icoeff", "dcoeff",
                                                "scale_sw", "scale_isw", "scale_dop", "scale_pol", "gravity_scale",
                                                "thomson_scale")])


_dp = ctypes.POINTER(ctypes.c_double)


class CTableView(ctypes.Structure):
    _fields_ = ([(n, ctypes.c_int) for n in ("n_k", "n_tau", "n_tab", "n_q")] +
                [(n, ctypes.c_double) for n in ("L0", "dlna", "tau0", "z_reio", "lna_tc", "N_massless", "Neff",
                                                "R_nu")] +
                [(n, _dp) for n in ("k", "lna_start", "lna_src", "tau_src", "chi_src", "w_src", "xe", "tm", "ln_dk",
                                    "kappa", "ln_cs2", "ln_tau", "M_ln_dk", "M_kappa", "M_ln_cs2", "M_ln_tau", "q",
                                    "W")] +
                [(n, ctypes.c_double) for n in ("rt_g0", "rt_ur0", "rt_c0", "rt_b0", "rt_L", "pref_ncdm", "m_over_T",
                                                "H0", "tau_star", "chi_star")] +
                [("lens_w", _dp)])


_vp = ctypes.c_void_p


class CServerOpts(ctypes.Structure):
    _fields_ = [("n_workers", ctypes.c_int), ("n_streams", ctypes.c_int), ("max_batch", ctypes.c_int),
                ("hbm_budget_bytes", ctypes.c_size_t)]


class CRequestTimes(ctypes.Structure):
    _fields_ = [("submit", ctypes.c_double), ("tables_ready", ctypes.c_double), ("launched", ctypes.c_double),
                ("done", ctypes.c_double), ("batch_size", ctypes.c_int)]


def _declare(lib):
    lib.cmb_defaults.argtypes = [ctypes.POINTER(CCosmo), ctypes.POINTER(CPrec)]
    lib.cmb_last_error.restype = ctypes.c_char_p
    lib.cmb_tables_build.argtypes = [ctypes.POINTER(CCosmo), ctypes.POINTER(CPrec), _dp, ctypes.c_int, ctypes.c_int,
                                      ctypes.POINTER(_vp)]
    lib.cmb_tables_destroy.argtypes = [_vp]
    lib.cmb_tables_destroy.restype = None
    lib.cmb_tables_export.argtypes = [_vp, ctypes.POINTER(CTableView)]
    lib.cmb_ctx_create.argtypes = [ctypes.c_int, ctypes.c_size_t, ctypes.POINTER(_vp)]
    lib.cmb_ctx_destroy.argtypes = [_vp]
    lib.cmb_ctx_destroy.restype = None
    lib.cmb_solve_workspace_bytes.argtypes = [ctypes.POINTER(_vp), ctypes.c_int]
    lib.cmb_solve_workspace_bytes.restype = ctypes.c_size_t
    lib.cmb_perturb.argtypes = [_vp, ctypes.POINTER(_vp), ctypes.c_int, _vp, _vp, _vp, _vp]
    lib.cmb_perturb_pk.argtypes = [_vp, ctypes.POINTER(_vp), ctypes.c_int, _vp, _vp, _vp, _vp, _vp]
    lib.cmb_transfer_kgrid.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, _dp, ctypes.c_int]
    lib.cmb_spectra_on_grid.argtypes = [_vp, ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int, _vp, _dp, ctypes.c_int,
                                        _vp, _vp, _vp, _vp]
    lib.cmb_los.argtypes = [_vp, ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int, _vp, _vp, _vp]
    lib.cmb_bessel3_table.argtypes = [_vp, ctypes.c_int, _dp, _dp, _dp]
    lib.cmb_perturb_matter.argtypes = [_vp, ctypes.POINTER(_vp), ctypes.c_int, _vp, _vp, _vp, _vp, _vp, _vp]
    lib.cmb_lensing_potential.argtypes = [_vp, ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int, _vp, _vp, _vp]
    lib.cmb_lensed_cl.argtypes = [_vp, ctypes.c_int, ctypes.c_int, _vp, _vp, ctypes.c_int, ctypes.c_int, _vp, _vp]
    lib.cmb_perturb_record.argtypes = [_vp, ctypes.POINTER(_vp), ctypes.c_int, _vp, _vp, _vp, _vp, _vp, ctypes.c_int,
                                       _vp]
    lib.cmb_perturb_replay.argtypes = [_vp, ctypes.POINTER(_vp), ctypes.c_int, _vp, _vp, ctypes.c_int, _vp, _vp, _vp,
                                       _vp]
    lib.cmb_perturb_checkpoint.argtypes = [_vp, ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int, _vp, _vp,
                                           ctypes.c_int, ctypes.c_int, _vp, ctypes.c_int, _vp, _vp, _vp, _vp]
    lib.cmb_perturb_segment.argtypes = [_vp, ctypes.POINTER(_vp), ctypes.c_int, _vp, _vp, ctypes.c_int, ctypes.c_int,
                                        _vp, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp, _vp]
    lib.cmb_spectra_adjoint.argtypes = [_vp, ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int, _vp, _vp, _vp, _vp]
    lib.cmb_state_rows.argtypes = [_vp]
    lib.cmb_sources_adjoint.argtypes = [_vp, ctypes.POINTER(_vp), ctypes.c_int, _vp, _vp, _vp]
    lib.cmb_jacobian.argtypes = [_vp, ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                 _vp, _vp, _vp, _vp]
    lib.cmb_gradient.argtypes = [_vp, ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int, _vp, ctypes.c_double, _vp, _vp,
                                 _vp, _vp, _vp]
    lib.cmb_los_bessel3.argtypes = [_vp, ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int, _vp, _vp, _vp]
    lib.cmb_cl.argtypes = [_vp, ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int, _vp, _vp, _vp]
    lib.cmb_solve.argtypes = [_vp, ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int, _vp, _vp, _vp, _vp, _vp, _vp]
    lib.cmb_solve_noalloc.argtypes = [ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int, _vp, _vp, _vp, _vp]
    lib.cmb_noalloc_scratch_bytes.argtypes = []
    lib.cmb_noalloc_scratch_bytes.restype = ctypes.c_size_t
    lib.cmb_server_create.argtypes = [ctypes.c_int, ctypes.POINTER(CServerOpts), ctypes.POINTER(_vp)]
    lib.cmb_server_submit.argtypes = [_vp, ctypes.POINTER(CCosmo), ctypes.POINTER(CPrec), _dp, ctypes.c_int,
                                      ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_uint64)]
    lib.cmb_server_wait.argtypes = [_vp, ctypes.c_uint64, ctypes.c_double, _dp, ctypes.POINTER(ctypes.c_int32),
                                    ctypes.POINTER(CRequestTimes)]
    lib.cmb_server_destroy.argtypes = [_vp]
    lib.cmb_server_destroy.restype = None
    lib.cmb_server_selftest_arena.argtypes = [ctypes.c_uint, ctypes.c_int]


def _load():
    if not os.path.exists(LIB_PATH):
        return _MissingLibrary()
    lib = ctypes.CDLL(LIB_PATH)
    missing = [f for f in EXPORTS if not hasattr(lib, f)]
    if missing:
        return _MissingLibrary(f"out of date (lacks {', '.join(missing)})")
    _declare(lib)
    return lib


_lib = _load()


def _check(rc: int, where: str):
    if rc != CMB_OK:
        raise CmbError(rc, where)


def abi_version() -> int:
    return _lib.cmb_abi_version()


def defaults():
    """(cosmo dict, prec dict) with the paper's defaults (App. A.2)."""
    c, p = CCosmo(), CPrec()
    _check(_lib.cmb_defaults(ctypes.byref(c), ctypes.byref(p)), "cmb_defaults")
    return {n: getattr(c, n) for n, _ in CCosmo._fields_}, {n: getattr(p, n) for n, _ in CPrec._fields_}


def _cosmo_struct(c: dict) -> CCosmo:
    d, _ = defaults()
    d.update({k: v for k, v in c.items() if k in d})
    # map workload key names
    if "z_reio" in c:
        d["z_reio"] = c["z_reio"]
    s = CCosmo()
    for n, _ in CCosmo._fields_:
        setattr(s, n, float(d[n]))
    return s


def _prec_struct(p: dict) -> CPrec:
    _, d = defaults()
    d.update({k: v for k, v in p.items() if k in d})
    s = CPrec()
    for n, t in CPrec._fields_:
        setattr(s, n, int(d[n]) if t is ctypes.c_int else float(d[n]))
    return s


class Tables:
    """Host tables of one cosmology (cmb_tables_build)."""

    def __init__(self, cosmo: dict, prec: dict, k, n_tau: int):
        self.cosmo = dict(cosmo)
        self.prec = dict(prec)
        k = np.ascontiguousarray(k, dtype=np.float64)
        self.k = k
        self.n_tau = int(n_tau)
        h = _vp()
        cs, ps = _cosmo_struct(cosmo), _prec_struct(prec)
        _check(_lib.cmb_tables_build(ctypes.byref(cs), ctypes.byref(ps), k.ctypes.data_as(_dp), len(k), int(n_tau),
                                     ctypes.byref(h)), "cmb_tables_build")
        self._h = h

    @property
    def handle(self):
        return self._h

    def state_rows(self) -> int:
        """Rows of one mode's perturbation state (cmb_state_rows)."""
        n = int(_lib.cmb_state_rows(self.handle))
        if n <= 0:
            _check(-n if n < 0 else 1, "cmb_state_rows")
        return n

    def export(self) -> dict:
        v = CTableView()
        _check(_lib.cmb_tables_export(self._h, ctypes.byref(v)), "cmb_tables_export")
        n1 = v.n_tab + 1

        def arr(ptr, n):
            return np.ctypeslib.as_array(ptr, shape=(n,)).copy() if n else np.zeros(0)

        out = {f: getattr(v, f) for f in ("n_k", "n_tau", "n_tab", "n_q", "L0", "dlna", "tau0", "z_reio", "lna_tc",
                                          "N_massless", "Neff", "R_nu", "rt_g0", "rt_ur0", "rt_c0", "rt_b0", "rt_L",
                                          "pref_ncdm", "m_over_T", "H0", "tau_star", "chi_star")}
        for f in ("k", "lna_start"):
            out[f] = arr(getattr(v, f), v.n_k)
        for f in ("lna_src", "tau_src", "chi_src", "w_src", "lens_w"):
            out[f] = arr(getattr(v, f), v.n_tau)
        for f in ("xe", "tm", "ln_dk", "kappa", "ln_cs2", "ln_tau", "M_ln_dk", "M_kappa", "M_ln_cs2", "M_ln_tau"):
            out[f] = arr(getattr(v, f), n1)
        for f in ("q", "W"):
            out[f] = arr(getattr(v, f), v.n_q)
        return out

    def __del__(self):
        h = getattr(self, "_h", None)
        lib = globals().get("_lib")  # None while the interpreter shuts down
        if h is not None and h.value and lib is not None:
            lib.cmb_tables_destroy(h)
            self._h = None


def build_tables(cosmo: dict, prec: dict, k, n_tau: int) -> Tables:
    return Tables(cosmo, prec, k, n_tau)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(int(stream))


def _handles(tabs):
    arr = (_vp * len(tabs))(*[t.handle for t in tabs])
    return arr


class Context:
    """Device context (cmb_ctx_create): one HIP device, a workspace budget."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        h = _vp()
        _check(_lib.cmb_ctx_create(int(device), int(hbm_budget_bytes), ctypes.byref(h)), "cmb_ctx_create")
        self._h = h
        self.device = device

    def close(self):
        lib = globals().get("_lib")  # None while the interpreter shuts down
        if getattr(self, "_h", None) is not None and self._h.value and lib is not None:
            lib.cmb_ctx_destroy(self._h)
        self._h = None

    def __del__(self):
        self.close()

    def perturb(self, tabs, S, status, nsteps=None, stream=None):
        hs = _handles(tabs)
        _check(_lib.cmb_perturb(self._h, hs, len(tabs), _ptr(S), _ptr(status), _ptr(nsteps), _stream(stream)),
               "cmb_perturb")

    def perturb_pk(self, tabs, S, status, Pk, nsteps=None, stream=None):
        """cmb_perturb plus the matter power spectrum today into Pk[n_cosmo][n_k]."""
        hs = _handles(tabs)
        _check(_lib.cmb_perturb_pk(self._h, hs, len(tabs), _ptr(S), _ptr(status), _ptr(nsteps), _ptr(Pk),
                                   _stream(stream)), "cmb_perturb_pk")

    def spectra_on_grid(self, tabs, ell_max, S, kt, St, Delta, Cl, stream=None):
        """Sources interpolated onto the transfer grid kt, then projection and
        k quadrature there (cmb_spectra_on_grid)."""
        hs = _handles(tabs)
        kt = np.ascontiguousarray(kt, dtype=np.float64)
        _check(_lib.cmb_spectra_on_grid(self._h, hs, len(tabs), int(ell_max), _ptr(S), kt.ctypes.data_as(_dp),
                                        len(kt), _ptr(St), _ptr(Delta), _ptr(Cl), _stream(stream)),
               "cmb_spectra_on_grid")

    def los(self, tabs, ell_max, S, Delta, stream=None):
        hs = _handles(tabs)
        _check(_lib.cmb_los(self._h, hs, len(tabs), int(ell_max), _ptr(S), _ptr(Delta), _stream(stream)), "cmb_los")

    def perturb_matter(self, tabs, S, status, Pk=None, Dm=None, nsteps=None, stream=None):
        """cmb_perturb plus P(k) today and/or delta_m at the output times."""
        hs = _handles(tabs)
        _check(_lib.cmb_perturb_matter(self._h, hs, len(tabs), _ptr(S), _ptr(status), _ptr(nsteps), _ptr(Pk),
                                       _ptr(Dm), _stream(stream)), "cmb_perturb_matter")

    def lensing_potential(self, tabs, ell_max, Dm, Clpp, stream=None):
        """Limber C_l^psipsi from delta_m (cmb_lensing_potential)."""
        hs = _handles(tabs)
        _check(_lib.cmb_lensing_potential(self._h, hs, len(tabs), int(ell_max), _ptr(Dm), _ptr(Clpp),
                                          _stream(stream)), "cmb_lensing_potential")

    def perturb_record(self, tabs, S, status, hist, hist_n, nsteps=None, stream=None):
        """cmb_perturb recording the accepted steps into hist[n][n_k][cap], hist_n[n][n_k]."""
        hs = _handles(tabs)
        _check(_lib.cmb_perturb_record(self._h, hs, len(tabs), _ptr(S), _ptr(status), _ptr(nsteps), _ptr(hist),
                                       _ptr(hist_n), int(hist.shape[-1]), _stream(stream)), "cmb_perturb_record")

    def perturb_replay(self, tabs, hist, hist_n, S, status, nsteps=None, stream=None):
        """Integrate every mode on its recorded steps (cmb_perturb_replay)."""
        hs = _handles(tabs)
        _check(_lib.cmb_perturb_replay(self._h, hs, len(tabs), _ptr(hist), _ptr(hist_n), int(hist.shape[-1]),
                                       _ptr(S), _ptr(status), _ptr(nsteps), _stream(stream)), "cmb_perturb_replay")

    def perturb_checkpoint(self, tabs, hist, hist_n, every, ck, S, status, nsteps=None, replay=False, stream=None):
        """Record (replay=False) or replay the step histories and write the
        trajectory checkpoints ck [n][n_k][ck_cap][1 + 2 N] every `every`
        accepted steps (cmb_perturb_checkpoint)."""
        hs = _handles(tabs)
        _check(_lib.cmb_perturb_checkpoint(self._h, hs, len(tabs), 1 if replay else 0, _ptr(hist), _ptr(hist_n),
                                           int(hist.shape[-1]), int(every), _ptr(ck), int(ck.shape[-2]), _ptr(S),
                                           _ptr(status), _ptr(nsteps), _stream(stream)), "cmb_perturb_checkpoint")

    def perturb_segment(self, tabs, hist, hist_n, every, ck, seg, S, status, nsteps=None, stream=None):
        """Replay segment seg (accepted steps seg*every+1 .. (seg+1)*every) of
        every mode from its checkpoint, writing only that segment's outputs
        into S (cmb_perturb_segment)."""
        hs = _handles(tabs)
        _check(_lib.cmb_perturb_segment(self._h, hs, len(tabs), _ptr(hist), _ptr(hist_n), int(hist.shape[-1]),
                                        int(every), _ptr(ck), int(ck.shape[-2]), int(seg), _ptr(S), _ptr(status),
                                        _ptr(nsteps), _stream(stream)), "cmb_perturb_segment")

    def spectra_adjoint(self, tabs, ell_max, Delta, gCl, gS, stream=None):
        """dL/dS from dL/dC_l through the transposed quadrature and projection."""
        hs = _handles(tabs)
        _check(_lib.cmb_spectra_adjoint(self._h, hs, len(tabs), int(ell_max), _ptr(Delta), _ptr(gCl), _ptr(gS),
                                        _stream(stream)), "cmb_spectra_adjoint")

    def sources_adjoint(self, tabs, gS, gY, stream=None):
        """dL/dy [n][n_k][n_tau][state_rows] from dL/dS [n][n_k][3][n_tau]
        (cmb_sources_adjoint)."""
        hs = _handles(tabs)
        _check(_lib.cmb_sources_adjoint(self._h, hs, len(tabs), _ptr(gS), _ptr(gY), _stream(stream)),
               "cmb_sources_adjoint")

    def jacobian(self, tabs, ell_max, Cl, J, status, rel=1e-4, order=4, stream=None):
        """C_l and dC_l/d(h, omega_b, omega_cdm, ln A_s, n_s, tau_reio) (cmb_jacobian)."""
        hs = _handles(tabs)
        _check(_lib.cmb_jacobian(self._h, hs, len(tabs), int(ell_max), float(rel), int(order), _ptr(Cl), _ptr(J),
                                 _ptr(status), _stream(stream)), "cmb_jacobian")

    def gradient(self, tabs, ell_max, gCl, Cl, grad, status, rel=1e-4, dLdy0=None, stream=None):
        """C_l and dL/d(h, omega_b, omega_cdm, ln A_s, n_s, tau_reio) for
        L = sum dL/dC_l C_l by the discrete adjoint (cmb_gradient)."""
        hs = _handles(tabs)
        _check(_lib.cmb_gradient(self._h, hs, len(tabs), int(ell_max), _ptr(gCl), float(rel), _ptr(Cl), _ptr(grad),
                                 _ptr(status), _ptr(dLdy0), _stream(stream)), "cmb_gradient")

    def lensed_cl(self, Cl, Clpp, ell_max, Cll, n_mu=None, stream=None):
        """Lensed TT, TE, EE, BB [n][4][ell_max+1] from unlensed Cl[n][3][L+1]
        and Clpp[n][L+1] (cmb_lensed_cl); n_mu defaults to L + ell_max/2 + 200."""
        n, L = int(Cl.shape[0]), int(Cl.shape[2]) - 1
        if n_mu is None:
            n_mu = L + ell_max // 2 + 200
        _check(_lib.cmb_lensed_cl(self._h, n, L, _ptr(Cl), _ptr(Clpp), int(ell_max), int(n_mu), _ptr(Cll),
                                  _stream(stream)), "cmb_lensed_cl")

    def los_bessel3(self, tabs, ell_max, S, Delta, stream=None):
        """cmb_los with the three-region Bessel scheme (cmb_los_bessel3)."""
        hs = _handles(tabs)
        _check(_lib.cmb_los_bessel3(self._h, hs, len(tabs), int(ell_max), _ptr(S), _ptr(Delta), _stream(stream)),
               "cmb_los_bessel3")

    def bessel3_table(self, ell_max, samples=True):
        """The context's three-region Bessel table for 1 <= l <= ell_max:
        (x_start, x_5, samples[l-1][5000] or None)."""
        xs, x5 = np.zeros(ell_max), np.zeros(ell_max)
        tab = np.zeros((ell_max, 5000)) if samples else None
        _check(_lib.cmb_bessel3_table(self._h, int(ell_max), xs.ctypes.data_as(_dp), x5.ctypes.data_as(_dp),
                                      tab.ctypes.data_as(_dp) if samples else None), "cmb_bessel3_table")
        return xs, x5, tab

    def cl(self, tabs, ell_max, Delta, Cl, stream=None):
        hs = _handles(tabs)
        _check(_lib.cmb_cl(self._h, hs, len(tabs), int(ell_max), _ptr(Delta), _ptr(Cl), _stream(stream)), "cmb_cl")

    def solve(self, tabs, ell_max, Cl, status, S=None, Delta=None, nsteps=None, stream=None):
        hs = _handles(tabs)
        _check(_lib.cmb_solve(self._h, hs, len(tabs), int(ell_max), _ptr(S), _ptr(Delta), _ptr(Cl), _ptr(status),
                              _ptr(nsteps), _stream(stream)), "cmb_solve")


def workspace_bytes(tabs) -> int:
    return int(_lib.cmb_solve_workspace_bytes(_handles(tabs), len(tabs)))


def solve_noalloc(tabs, ell_max, Cl, status, nsteps=None, stream=None):
    """cmb_solve_noalloc: the whole path on the current device with every
    intermediate in the library's fixed device array (no allocation)."""
    hs = _handles(tabs)
    _check(_lib.cmb_solve_noalloc(hs, len(tabs), int(ell_max), _ptr(Cl), _ptr(status), _ptr(nsteps),
                                  _stream(stream)), "cmb_solve_noalloc")


def noalloc_scratch_bytes() -> int:
    return int(_lib.cmb_noalloc_scratch_bytes())


def alloc_outputs(tabs, ell_max: int, device: str = "cuda:0", keep_S: bool = True, keep_Delta: bool = True):
    """torch device tensors for one batch, laid out as include/cmbhip.h states."""
    import torch
    B = len(tabs)
    n_k, n_tau = len(tabs[0].k), tabs[0].n_tau
    out = {
        "Cl": torch.empty((B, 3, ell_max + 1), dtype=torch.float64, device=device),
        "status": torch.empty((B, n_k), dtype=torch.int32, device=device),
        "nsteps": torch.empty((B, n_k), dtype=torch.int32, device=device),
    }
    out["S"] = torch.empty((B, n_k, 3, n_tau), dtype=torch.float64, device=device) if keep_S else None
    out["Delta"] = torch.empty((B, 2, n_k, ell_max - 1), dtype=torch.float64, device=device) if keep_Delta else None
    return out


def solve_batch(ctx: Context, tabs, ell_max: int, keep_S: bool = True, keep_Delta: bool = True, stream=None):
    """Run the whole path for a batch of tables; returns torch tensors."""
    dev = f"cuda:{ctx.device}"
    out = alloc_outputs(tabs, ell_max, dev, keep_S, keep_Delta)
    ctx.solve(tabs, ell_max, out["Cl"], out["status"], S=out["S"], Delta=out["Delta"], nsteps=out["nsteps"],
              stream=stream)
    return out


class Server:
    """Continuous-batching runtime (cmb_server_*): submit spectrum requests
    from the host, wait for their C_ell.  All requests share the hierarchy
    options of their prec dicts."""

    def __init__(self, device: int = 0, n_workers: int = 0, n_streams: int = 0, max_batch: int = 0,
                 hbm_budget_bytes: int = 0):
        o = CServerOpts(int(n_workers), int(n_streams), int(max_batch), int(hbm_budget_bytes))
        h = _vp()
        _check(_lib.cmb_server_create(int(device), ctypes.byref(o), ctypes.byref(h)), "cmb_server_create")
        self._h = h
        self._shape = {}

    def submit(self, cosmo: dict, prec: dict, k, n_tau: int, ell_max: int) -> int:
        k = np.ascontiguousarray(k, dtype=np.float64)
        cs, ps = _cosmo_struct(cosmo), _prec_struct(prec)
        t = ctypes.c_uint64()
        _check(_lib.cmb_server_submit(self._h, ctypes.byref(cs), ctypes.byref(ps), k.ctypes.data_as(_dp), len(k),
                                      int(n_tau), int(ell_max), ctypes.byref(t)), "cmb_server_submit")
        self._shape[t.value] = (len(k), int(ell_max))
        return t.value

    def wait(self, ticket: int, timeout_s: float = -1.0):
        """(C_ell[3][ell_max+1], status[n_k], times dict); raises CmbError on a
        failed request, TimeoutError on timeout."""
        n_k, ell_max = self._shape[ticket]
        Cl = np.zeros((3, ell_max + 1))
        st = np.zeros(n_k, dtype=np.int32)
        tm = CRequestTimes()
        rc = _lib.cmb_server_wait(self._h, ctypes.c_uint64(ticket), float(timeout_s), Cl.ctypes.data_as(_dp),
                                  st.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(tm))
        if rc == -1:
            raise TimeoutError(f"request {ticket} not done after {timeout_s} s")
        del self._shape[ticket]
        _check(rc, "cmb_server_wait")
        times = {n: getattr(tm, n) for n, _ in CRequestTimes._fields_}
        return Cl, st, times

    def close(self):
        lib = globals().get("_lib")  # None while the interpreter shuts down
        if getattr(self, "_h", None) is not None and self._h.value and lib is not None:
            lib.cmb_server_destroy(self._h)
        self._h = None

    def __del__(self):
        self.close()


def server_selftest_arena(seed: int = 1, n_ops: int = 20000) -> int:
    """Host self-test of the server's device-arena allocator (no GPU)."""
    return int(_lib.cmb_server_selftest_arena(int(seed), int(n_ops)))


def transfer_kgrid(ell_max: int, k_lo: float, k_hi: float) -> np.ndarray:
    """The transfer k-grid of cmb_transfer_kgrid."""
    n = _lib.cmb_transfer_kgrid(int(ell_max), float(k_lo), float(k_hi), None, 0)
    if n < 0:
        raise CmbError(-n, "cmb_transfer_kgrid")
    out = np.zeros(n)
    _lib.cmb_transfer_kgrid(int(ell_max), float(k_lo), float(k_hi), out.ctypes.data_as(_dp), n)
    return out
