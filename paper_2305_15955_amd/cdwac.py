"""ctypes binding of libcdwac.so (the C ABI in include/cdwac.h).

Argument marshalling only: every step of the self-energy path runs in the
library's HIP kernels.  PyTorch provides device memory and the stream.  The
functions keep the C names; ``Cdwac`` bundles a context with the device
copies of one system for convenience.

Importing this module never falls back to anything: if the library is not
built, or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes
import math
import os
import re
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcdwac.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "cdwac.h")

CDWAC_OK, CDWAC_EINVAL, CDWAC_ENOMEM, CDWAC_EHIP, CDWAC_ENOTPD, CDWAC_ESTATE = 0, -1, -2, -3, -4, -5
CDWAC_EFACT = -6
CDWAC_WNOROOT = 1
CDWAC_P64, CDWAC_B16X3, CDWAC_B16, CDWAC_F16X3, CDWAC_F16 = 0, 1, 2, 3, 4
FLAG_NOROOT, FLAG_FALLBACK, FLAG_MLP_ACCEPTED = 1, 2, 4
MLP_NPARAM = 4801
PREC = {"p64": CDWAC_P64, "b16x3": CDWAC_B16X3, "b16": CDWAC_B16, "f16x3": CDWAC_F16X3, "f16": CDWAC_F16}
# Skeleton-node tolerance (freq_rank_tol) of each 16-bit mode, set at the W
# error the mode's own contractions leave on the imaginary axis, so that the
# frequency interpolation adds nothing visible: one fp16 product 1.6e-6 of
# max|W|, the fp16 split 2e-8 (measured against the FP64 path at N_aux = 5000).
# The bf16 modes, not measured, take the fp16 values.
SKELETON_TOL = {"f16": 1e-6, "b16": 1e-6, "f16x3": 1e-8, "b16x3": 1e-8, "p64": 0.0}

_i32p = ctypes.POINTER(ctypes.c_int32)
_f64p = ctypes.POINTER(ctypes.c_double)
_f32p = ctypes.POINTER(ctypes.c_float)
_vp = ctypes.c_void_p


class CdwacSystem(ctypes.Structure):
    _fields_ = [("n_mo", ctypes.c_int32), ("n_occ", ctypes.c_int32), ("n_aux", ctypes.c_int32),
                ("n_states", ctypes.c_int32), ("state_idx", _i32p), ("eps", _f64p), ("vxc", _f64p),
                ("o_ia", _vp), ("o_nm", _vp), ("spin", ctypes.c_double),
                ("eps_fermi", ctypes.c_double)]


class CdwacParams(ctypes.Structure):
    _fields_ = [("n_freq", ctypes.c_int32), ("freq", _f64p), ("weight", _f64p),
                ("n_ref_im", ctypes.c_int32), ("ref_im_idx", _i32p), ("n_ref_re", ctypes.c_int32),
                ("ref_re", _f64p), ("eta_ref", ctypes.c_double), ("eta", ctypes.c_double),
                ("pade_tol", ctypes.c_double), ("win_lo", _f64p), ("win_hi", _f64p),
                ("qp_tol", ctypes.c_double), ("qp_maxit", ctypes.c_int32), ("prec", ctypes.c_int32),
                ("use_mlp_seed", ctypes.c_int32), ("mlp_accept", ctypes.c_double),
                ("freq_rank_tol", ctypes.c_double), ("fit_all", ctypes.c_int32),
                ("near_real_f64", ctypes.c_int32), ("quad_limit", ctypes.c_int32)]


class CdwacStateOut(ctypes.Structure):
    _fields_ = [("qp", ctypes.c_double), ("z", ctypes.c_double), ("sigma_x", ctypes.c_double),
                ("sigma_c", ctypes.c_double), ("residual", ctypes.c_double),
                ("n_evals", ctypes.c_int32), ("flags", ctypes.c_int32), ("n_rounds", ctypes.c_int32)]


class CdwacError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"cdwac error {code}: {msg}")
        self.code = code


_SIGNATURES = {
    "cdwac_ctx_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, _vp]),
    "cdwac_ctx_destroy": (None, [_vp]),
    "cdwac_last_error": (ctypes.c_char_p, [_vp]),
    "cdwac_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(CdwacSystem), ctypes.POINTER(CdwacParams)]),
    "cdwac_set_workspace": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t]),
    "cdwac_prepare": (ctypes.c_int, [_vp, ctypes.POINTER(CdwacSystem), ctypes.POINTER(CdwacParams)]),
    "cdwac_qp": (ctypes.c_int, [_vp, _f64p, ctypes.POINTER(CdwacStateOut)]),
    "cdwac_set_g_energies": (ctypes.c_int, [_vp, _f64p, ctypes.c_double]),
    "cdwac_qp_hedin": (ctypes.c_int, [_vp, _f64p, ctypes.POINTER(CdwacStateOut), _f64p]),
    "cdwac_evgw": (ctypes.c_int, [_vp, ctypes.POINTER(CdwacSystem), ctypes.POINTER(CdwacParams), ctypes.c_int32,
                                  ctypes.c_int32, ctypes.c_double, _f64p, _i32p, ctypes.POINTER(CdwacStateOut)]),
    "cdwac_sigma_cd": (ctypes.c_int, [_vp, ctypes.POINTER(CdwacSystem), ctypes.POINTER(CdwacParams),
                                      ctypes.c_int32, ctypes.c_double, _f64p, _i32p]),
    "cdwac_solve_batch": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.POINTER(CdwacSystem),
                                         ctypes.POINTER(CdwacParams), ctypes.POINTER(CdwacStateOut)]),
    "cdwac_solve": (ctypes.c_int, [_vp, ctypes.POINTER(CdwacSystem), ctypes.POINTER(CdwacParams),
                                   ctypes.POINTER(CdwacStateOut)]),
    "cdwac_sigma": (ctypes.c_int, [_vp, ctypes.c_int32, _vp, _vp, _vp, _vp]),
    "cdwac_w_table": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "cdwac_fit_ranges": (ctypes.c_int, [_vp, _i32p, _i32p, _i32p]),
    "cdwac_polarizability": (ctypes.c_int, [_vp, ctypes.POINTER(CdwacSystem), ctypes.c_int32, ctypes.c_int32,
                                            _f64p, _f64p, _vp, _vp]),
    "cdwac_pade_fit_eval": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp, ctypes.c_double,
                                           ctypes.c_int32, _vp, _vp, _vp]),
    "cdwac_pade_fit_eval_noalloc": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp,
                                                   ctypes.c_double, ctypes.c_int32, _vp, _vp, _vp]),
    "cdwac_set_timing": (ctypes.c_int, [_vp, ctypes.c_int]),
    "cdwac_get_timing": (ctypes.c_int, [_vp, _f64p, ctypes.c_int32]),
    "cdwac_freq_decomposition": (ctypes.c_int, [ctypes.c_int32, _f64p, ctypes.c_double, ctypes.c_double,
                                                 ctypes.c_double, ctypes.POINTER(ctypes.c_int32),
                                                 ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                                 _f64p]),
    "cdwac_spectral": (ctypes.c_int, [_vp, ctypes.c_int32, _vp, _f64p, _vp, _vp, _vp]),
    "cdwac_plane_counts": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    "cdwac_get_timing_segments": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32]),
    "cdwac_inversion_residual": (ctypes.c_int, [_vp, _f64p, ctypes.POINTER(ctypes.c_int32)]),
    "cdwac_mlp_set_model": (ctypes.c_int, [_vp, _f32p, _f32p, _f32p, ctypes.c_float, ctypes.c_float]),
    "cdwac_mlp_forward": (ctypes.c_int, [_vp, _vp, ctypes.c_int32, _vp, _vp]),
    "cdwac_mlp_grad": (ctypes.c_int, [_vp, _vp, ctypes.c_int32, _vp, _vp, _vp, _vp]),
    "cdwac_mlp_adam": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, ctypes.c_int32, ctypes.c_float, ctypes.c_float,
                                      ctypes.c_float, ctypes.c_float]),
    "cdwac_mlp_train": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.c_int32, _vp, _vp, ctypes.c_int32,
                                       ctypes.c_int32, ctypes.c_float, ctypes.c_uint64, _f32p]),
}

_lib = None


def load_library(path: str = LIB_PATH):
    """Loads libcdwac.so and declares every entry point; raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built (run paper_2305_15955_amd/build.py)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def freq_decomposition(freq, omega_lo: float, omega_hi: float, tol: float):
    """Host-only skeleton of the imaginary nodes (cdwac_freq_decomposition):
    returns (skel, rest, T) with 1/(w_rest[r]^2 + O^2) ~= sum_s T[r, s] / (w_skel[s]^2 + O^2)
    for O in [omega_lo, omega_hi]."""
    lib = load_library()
    w = np.ascontiguousarray(freq, np.float64)
    n = len(w)
    ns = ctypes.c_int32(0)
    skel = np.zeros(n, np.int32)
    rest = np.zeros(n, np.int32)
    T = np.zeros(n * n, np.float64)
    rc = lib.cdwac_freq_decomposition(n, _np_ptr(w, ctypes.c_double), float(omega_lo), float(omega_hi), float(tol),
                                      ctypes.byref(ns), _np_ptr(skel, ctypes.c_int32),
                                      _np_ptr(rest, ctypes.c_int32), _np_ptr(T, ctypes.c_double))
    if rc != 0:
        raise ValueError(f"cdwac_freq_decomposition failed ({rc})")
    k = ns.value
    return skel[:k].copy(), rest[:n - k].copy(), T[:(n - k) * k].reshape(n - k, k).copy()


def header_functions(path: str = HEADER):
    """Names of the functions declared in include/cdwac.h."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cdwac_[a-z0-9_]+)\s*\(", text)))


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def _np_ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _check(ctx, rc: int, allow_warn: bool = False):
    if rc == CDWAC_OK or (allow_warn and rc > 0):
        return rc
    lib = load_library()
    msg = lib.cdwac_last_error(ctx).decode() if ctx else ""
    raise CdwacError(rc, msg)


# ---------------------------------------------------------------------------
# Thin wrappers with the C names
# ---------------------------------------------------------------------------

def cdwac_ctx_create(device: int = 0, stream: Optional[int] = None):
    lib = load_library()
    h = _vp()
    rc = lib.cdwac_ctx_create(ctypes.byref(h), device, stream)
    if rc != CDWAC_OK:
        raise CdwacError(rc, "cannot create context")
    return h


def cdwac_ctx_destroy(ctx):
    load_library().cdwac_ctx_destroy(ctx)


class Cdwac:
    """A context plus the host/device arrays of one system and its settings.

    ``system``: an object with eps, n_occ, o_ia, o_nm, state_idx, spin
    (numpy arrays or torch tensors; the RI coefficients are moved to the GPU
    once).  All energies in Hartree.
    """

    def __init__(self, device: int = 0, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the CD-WAC library needs a HIP device")
        self.torch = torch
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        self.lib = load_library()
        self.ctx = cdwac_ctx_create(device, stream.cuda_stream)
        self._keep = []
        self.ws = None

    def close(self):
        if self.ctx:
            self.lib.cdwac_ctx_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- marshalling ------------------------------------------------------
    def _dev(self, a):
        t = self.torch
        if isinstance(a, t.Tensor):
            return a.to(self.device, dtype=t.float64).contiguous()
        return t.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(self.device)

    def make_system(self, system, vxc=None, eps_fermi=None, o_ia_dev=None, o_nm_dev=None):
        eps = np.ascontiguousarray(system.eps, np.float64)
        sidx = np.ascontiguousarray(system.state_idx, np.int32)
        o_ia = o_ia_dev if o_ia_dev is not None else self._dev(system.o_ia)
        o_nm = o_nm_dev if o_nm_dev is not None else self._dev(system.o_nm)
        vx = None if vxc is None else np.ascontiguousarray(vxc, np.float64)
        s = CdwacSystem(n_mo=len(eps), n_occ=int(system.n_occ), n_aux=int(o_ia.shape[0]),
                        n_states=len(sidx), state_idx=_np_ptr(sidx, ctypes.c_int32),
                        eps=_np_ptr(eps, ctypes.c_double),
                        vxc=None if vx is None else _np_ptr(vx, ctypes.c_double),
                        o_ia=_ptr(o_ia), o_nm=_ptr(o_nm), spin=float(getattr(system, "spin", 2.0)),
                        eps_fermi=math.nan if eps_fermi is None else float(eps_fermi))
        keep = (eps, sidx, vx, o_ia, o_nm)
        return s, keep

    @staticmethod
    def make_params(freq, weight, ref_im_idx, ref_re, win_lo, win_hi, eta=1e-3, eta_ref=1e-3,
                    pade_tol=1e-9, qp_tol=1e-10, qp_maxit=100, prec="p64", use_mlp_seed=False,
                    mlp_accept=0.0, freq_rank_tol=0.0, fit_all=False,
                    near_real_f64=False, quad_limit=False):
        arrs = dict(freq=np.ascontiguousarray(freq, np.float64),
                    weight=np.ascontiguousarray(weight, np.float64),
                    ref_im=np.ascontiguousarray(ref_im_idx, np.int32),
                    ref_re=np.ascontiguousarray(ref_re, np.float64),
                    lo=np.ascontiguousarray(win_lo, np.float64),
                    hi=np.ascontiguousarray(win_hi, np.float64))
        p = CdwacParams(n_freq=len(arrs["freq"]), freq=_np_ptr(arrs["freq"], ctypes.c_double),
                        weight=_np_ptr(arrs["weight"], ctypes.c_double),
                        n_ref_im=len(arrs["ref_im"]), ref_im_idx=_np_ptr(arrs["ref_im"], ctypes.c_int32),
                        n_ref_re=len(arrs["ref_re"]), ref_re=_np_ptr(arrs["ref_re"], ctypes.c_double),
                        eta_ref=eta_ref, eta=eta, pade_tol=pade_tol,
                        win_lo=_np_ptr(arrs["lo"], ctypes.c_double),
                        win_hi=_np_ptr(arrs["hi"], ctypes.c_double), qp_tol=qp_tol,
                        qp_maxit=qp_maxit, prec=PREC[prec] if isinstance(prec, str) else int(prec),
                        use_mlp_seed=int(bool(use_mlp_seed)), mlp_accept=mlp_accept,
                        freq_rank_tol=freq_rank_tol, fit_all=int(bool(fit_all)),
                        near_real_f64=int(bool(near_real_f64)), quad_limit=int(bool(quad_limit)))
        return p, arrs

    # -- entry points -----------------------------------------------------
    def cdwac_workspace_bytes(self, sysc, prm) -> int:
        return int(self.lib.cdwac_workspace_bytes(ctypes.byref(sysc), ctypes.byref(prm)))

    def cdwac_set_workspace(self, nbytes: int):
        t = self.torch
        self.ws = t.empty(int(nbytes) + 256, dtype=t.uint8, device=self.device)
        base = _ptr(self.ws)
        aligned = (base + 255) // 256 * 256
        _check(self.ctx, self.lib.cdwac_set_workspace(self.ctx, aligned, int(nbytes)))

    def cdwac_prepare(self, sysc, prm):
        _check(self.ctx, self.lib.cdwac_prepare(self.ctx, ctypes.byref(sysc), ctypes.byref(prm)))

    def cdwac_qp(self, n_states: int, vxc=None):
        out = (CdwacStateOut * n_states)()
        vx = None if vxc is None else np.ascontiguousarray(vxc, np.float64)
        rc = self.lib.cdwac_qp(self.ctx, None if vx is None else _np_ptr(vx, ctypes.c_double), out)
        _check(self.ctx, rc, allow_warn=True)
        return _outs(out)

    def cdwac_qp_hedin(self, n_states: int, vxc=None):
        """G_dH W0 roots -> (state results, the shifts dH_n used)."""
        out = (CdwacStateOut * n_states)()
        vx = None if vxc is None else np.ascontiguousarray(vxc, np.float64)
        dh = np.zeros(n_states, np.float64)
        rc = self.lib.cdwac_qp_hedin(self.ctx, None if vx is None else _np_ptr(vx, ctypes.c_double), out,
                                     _np_ptr(dh, ctypes.c_double))
        _check(self.ctx, rc, allow_warn=True)
        return _outs(out), dh

    def cdwac_solve(self, sysc, prm):
        out = (CdwacStateOut * sysc.n_states)()
        rc = self.lib.cdwac_solve(self.ctx, ctypes.byref(sysc), ctypes.byref(prm), out)
        _check(self.ctx, rc, allow_warn=True)
        return _outs(out)

    def cdwac_solve_batch(self, systems, params):
        """systems, params: lists of CdwacSystem / CdwacParams (one per system)
        -> list of per-system lists of state results."""
        n = len(systems)
        sa = (CdwacSystem * n)(*systems)
        pa = (CdwacParams * n)(*params)
        counts = [int(x.n_states) for x in systems]
        out = (CdwacStateOut * sum(counts))()
        rc = self.lib.cdwac_solve_batch(self.ctx, n, sa, pa, out)
        _check(self.ctx, rc, allow_warn=True)
        flat = _outs(out)
        res, k = [], 0
        for c in counts:
            res.append(flat[k:k + c])
            k += c
        return res

    def cdwac_set_g_energies(self, eps_g, eps_fermi=None):
        e = np.ascontiguousarray(eps_g, np.float64)
        _check(self.ctx, self.lib.cdwac_set_g_energies(self.ctx, _np_ptr(e, ctypes.c_double),
                                                       math.nan if eps_fermi is None else float(eps_fermi)))

    def cdwac_evgw(self, sysc, prm, mode: str = "evgw0", max_iter: int = 20, tol: float = 1e-8):
        """mode 'evgw0' (W from the KS energies) or 'evgw' (W rebuilt) ->
        (final energies [n_mo], QP solves done, last solve's state results)."""
        eps = np.zeros(sysc.n_mo, np.float64)
        nit = ctypes.c_int32(0)
        out = (CdwacStateOut * sysc.n_states)()
        rc = self.lib.cdwac_evgw(self.ctx, ctypes.byref(sysc), ctypes.byref(prm),
                                 {"evgw0": 0, "evgw": 1}[mode], int(max_iter), float(tol),
                                 _np_ptr(eps, ctypes.c_double), ctypes.byref(nit), out)
        _check(self.ctx, rc, allow_warn=True)
        return eps, int(nit.value), _outs(out)

    def cdwac_sigma_cd(self, sysc, prm, state: int, omega: float):
        """Full-CD Sigma_n(omega) -> (Sigma, R_n, I_n, residue count)."""
        out = np.zeros(3, np.float64)
        nr = ctypes.c_int32(0)
        _check(self.ctx, self.lib.cdwac_sigma_cd(self.ctx, ctypes.byref(sysc), ctypes.byref(prm), int(state),
                                                 float(omega), _np_ptr(out, ctypes.c_double), ctypes.byref(nr)))
        return float(out[0]), float(out[1]), float(out[2]), int(nr.value)

    def cdwac_sigma(self, omega, terms: bool = False):
        """omega: [n_states, n_omega] (Ha) -> Re Sigma (and I, R) as numpy."""
        t = self.torch
        om = self._dev(np.atleast_2d(omega))
        sig = t.empty_like(om)
        it = t.empty_like(om) if terms else None
        rt = t.empty_like(om) if terms else None
        _check(self.ctx, self.lib.cdwac_sigma(self.ctx, om.shape[1], _ptr(om), _ptr(sig), _ptr(it),
                                              _ptr(rt)))
        if terms:
            return sig.cpu().numpy(), it.cpu().numpy(), rt.cpu().numpy()
        return sig.cpu().numpy()

    def cdwac_spectral(self, omega, vxc=None, parts: bool = False):
        """omega: [n_states, n_omega] (Ha) -> A_n(omega) (and Re, Im Sigma) as numpy."""
        t = self.torch
        om = self._dev(np.atleast_2d(omega))
        spec = t.empty_like(om)
        sre = t.empty_like(om) if parts else None
        sim = t.empty_like(om) if parts else None
        vx = None if vxc is None else np.ascontiguousarray(vxc, np.float64)
        _check(self.ctx, self.lib.cdwac_spectral(self.ctx, om.shape[1], _ptr(om),
                                                 None if vx is None else _np_ptr(vx, ctypes.c_double),
                                                 _ptr(spec), _ptr(sre), _ptr(sim)))
        if parts:
            return spec.cpu().numpy(), sre.cpu().numpy(), sim.cpu().numpy()
        return spec.cpu().numpy()

    def cdwac_fit_ranges(self, n_states: int):
        m0 = np.zeros(n_states, np.int32)
        m1 = np.zeros(n_states, np.int32)
        nf = ctypes.c_int32(0)
        _check(self.ctx, self.lib.cdwac_fit_ranges(self.ctx, _np_ptr(m0, ctypes.c_int32),
                                                   _np_ptr(m1, ctypes.c_int32), ctypes.byref(nf)))
        return m0, m1, nf.value

    def cdwac_w_table(self, n_states: int, n_mo: int, n_freq: int, n_re: int):
        t = self.torch
        m0, m1, nfit = self.cdwac_fit_ranges(n_states)
        w_im = t.empty((n_states, n_mo, n_freq), dtype=t.float64, device=self.device)
        w_re = t.empty((max(nfit, 1), max(n_re, 1), 2), dtype=t.float64, device=self.device)
        sx = t.empty(n_states, dtype=t.float64, device=self.device)
        _check(self.ctx, self.lib.cdwac_w_table(self.ctx, _ptr(w_im), _ptr(w_re), _ptr(sx)))
        wr = w_re.cpu().numpy()
        wr = wr[..., 0] + 1j * wr[..., 1]
        return w_im.cpu().numpy(), wr[:nfit, :n_re], sx.cpu().numpy(), (m0, m1)

    def cdwac_polarizability(self, sysc, zs: Sequence[complex], prec="p64"):
        t = self.torch
        zs = [complex(z) for z in zs]
        zr = np.array([z.real for z in zs])
        zi = np.array([z.imag for z in zs])
        n = sysc.n_aux
        pr = t.empty((len(zs), n, n), dtype=t.float64, device=self.device)
        pi = t.empty((len(zs), n, n), dtype=t.float64, device=self.device)
        _check(self.ctx, self.lib.cdwac_polarizability(
            self.ctx, ctypes.byref(sysc), PREC[prec] if isinstance(prec, str) else int(prec), len(zs),
            _np_ptr(zr, ctypes.c_double), _np_ptr(zi, ctypes.c_double), _ptr(pr), _ptr(pi)))
        return pr.cpu().numpy() + 1j * pi.cpu().numpy()

    def cdwac_pade_fit_eval(self, u, w, tol, x):
        """u, w: complex [n_fit, n_pts]; x: complex [n_fit, n_x] (values of z^2)."""
        t = self.torch

        def c2(a):
            a = np.asarray(a, np.complex128)
            return self._dev(np.stack([a.real, a.imag], axis=-1))
        nf, npts = np.asarray(u).shape
        nx = np.asarray(x).shape[1]
        ud, wd, xd = c2(u), c2(w), c2(x)
        out = t.empty((nf, nx, 2), dtype=t.float64, device=self.device)
        nt = t.empty(nf, dtype=t.int32, device=self.device)
        _check(self.ctx, self.lib.cdwac_pade_fit_eval(self.ctx, nf, npts, _ptr(ud), _ptr(wd), float(tol), nx,
                                                      _ptr(xd), _ptr(out), _ptr(nt)))
        o = out.cpu().numpy()
        return o[..., 0] + 1j * o[..., 1], nt.cpu().numpy()

    def cdwac_pade_fit_eval_noalloc(self, u, w, tol, x):
        """cdwac_pade_fit_eval through the allocation-free entry point (the
        library's fixed scratch; n_fit * n_pts <= 524288)."""
        t = self.torch

        def c2(a):
            a = np.asarray(a, np.complex128)
            return self._dev(np.stack([a.real, a.imag], axis=-1))
        nf, npts = np.asarray(u).shape
        nx = np.asarray(x).shape[1]
        ud, wd, xd = c2(u), c2(w), c2(x)
        out = t.empty((nf, nx, 2), dtype=t.float64, device=self.device)
        nt = t.empty(nf, dtype=t.int32, device=self.device)
        _check(self.ctx, self.lib.cdwac_pade_fit_eval_noalloc(self.ctx, nf, npts, _ptr(ud), _ptr(wd), float(tol),
                                                              nx, _ptr(xd), _ptr(out), _ptr(nt)))
        o = out.cpu().numpy()
        return o[..., 0] + 1j * o[..., 1], nt.cpu().numpy()

    STAGES = ("staging", "polarizability", "sweep_inversion", "lambda_finalize", "w_contraction",
              "exchange_and_fits", "qp", "prescale")

    def cdwac_set_timing(self, on: bool = True):
        _check(self.ctx, self.lib.cdwac_set_timing(self.ctx, int(bool(on))))

    def cdwac_get_timing(self):
        ms = np.zeros(len(self.STAGES))
        _check(self.ctx, self.lib.cdwac_get_timing(self.ctx, _np_ptr(ms, ctypes.c_double), len(ms)))
        return dict(zip(self.STAGES, ms.tolist()))

    def cdwac_plane_counts(self):
        a, b = ctypes.c_int32(0), ctypes.c_int32(0)
        _check(self.ctx, self.lib.cdwac_plane_counts(self.ctx, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def cdwac_get_timing_segments(self):
        n = np.zeros(len(self.STAGES), np.int32)
        _check(self.ctx, self.lib.cdwac_get_timing_segments(self.ctx, _np_ptr(n, ctypes.c_int32), len(n)))
        return dict(zip(self.STAGES, n.tolist()))

    def cdwac_inversion_residual(self):
        """(largest sampled residual ratio of the last preparation's inversions, its matrix index)."""
        r, m = ctypes.c_double(0.0), ctypes.c_int32(-1)
        _check(self.ctx, self.lib.cdwac_inversion_residual(self.ctx, ctypes.byref(r), ctypes.byref(m)))
        return r.value, m.value

    # -- learned seed -------------------------------------------------------
    def cdwac_mlp_set_model(self, theta, mu, sd, out_mu: float, out_sd: float):
        th = np.ascontiguousarray(theta, np.float32)
        mu = np.ascontiguousarray(mu, np.float32)
        sd = np.ascontiguousarray(sd, np.float32)
        _check(self.ctx, self.lib.cdwac_mlp_set_model(self.ctx, _np_ptr(th, ctypes.c_float),
                                                      _np_ptr(mu, ctypes.c_float), _np_ptr(sd, ctypes.c_float),
                                                      float(out_mu), float(out_sd)))

    def _f32(self, a):
        t = self.torch
        if isinstance(a, t.Tensor):
            return a.to(self.device, dtype=t.float32).contiguous()
        return t.from_numpy(np.ascontiguousarray(a, np.float32)).to(self.device)

    def cdwac_mlp_forward(self, theta, x):
        th, xd = self._f32(theta), self._f32(x)
        y = self.torch.empty(xd.shape[0], dtype=self.torch.float32, device=self.device)
        _check(self.ctx, self.lib.cdwac_mlp_forward(self.ctx, _ptr(th), xd.shape[0], _ptr(xd), _ptr(y)))
        return y.cpu().numpy()

    def cdwac_mlp_grad(self, theta, x, tgt):
        th, xd, td = self._f32(theta), self._f32(x), self._f32(tgt)
        g = self.torch.empty(MLP_NPARAM, dtype=self.torch.float32, device=self.device)
        loss = self.torch.empty(1, dtype=self.torch.float32, device=self.device)
        _check(self.ctx, self.lib.cdwac_mlp_grad(self.ctx, _ptr(th), xd.shape[0], _ptr(xd), _ptr(td), _ptr(g),
                                                 _ptr(loss)))
        return float(loss.cpu()[0]), g.cpu().numpy()

    def cdwac_mlp_adam(self, theta, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        """In place on the given device tensors."""
        _check(self.ctx, self.lib.cdwac_mlp_adam(self.ctx, _ptr(theta), _ptr(grad), _ptr(m), _ptr(v), int(step),
                                                 float(lr), float(beta1), float(beta2), float(eps)))

    def cdwac_mlp_train(self, theta, x, tgt, epochs, batch, lr, seed=0):
        """Returns (trained theta as numpy, loss per epoch)."""
        t = self.torch
        th = self._f32(theta).clone()
        m = t.zeros_like(th)
        v = t.zeros_like(th)
        xd, td = self._f32(x), self._f32(tgt)
        curve = np.zeros(epochs, np.float32)
        _check(self.ctx, self.lib.cdwac_mlp_train(self.ctx, _ptr(th), _ptr(m), _ptr(v), xd.shape[0], _ptr(xd),
                                                  _ptr(td), int(epochs), int(batch), float(lr), int(seed),
                                                  _np_ptr(curve, ctypes.c_float)))
        return th.cpu().numpy(), curve


def _outs(out):
    return [dict(qp=o.qp, z=o.z, sigma_x=o.sigma_x, sigma_c=o.sigma_c, residual=o.residual,
                 n_evals=o.n_evals, flags=o.flags, n_rounds=o.n_rounds) for o in out]
