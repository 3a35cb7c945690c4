"""ctypes binding of libarche.so (C ABI in include/arche.h and
include/arche_kernels.h).  Argument marshalling only: every step of the SCF
path runs in the library's HIP kernels.  Device buffers for the kernel-level
calls come from PyTorch (``tensor.data_ptr()``), which is used here for device
memory and streams only.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libarche.so")

OK, EINVAL, ENOMEM, EHIP, ENOCONV, ESTATE = 0, -1, -2, -3, -4, -5
INIT_UNIFORM, INIT_ONE_CENTER, INIT_KEEP, INIT_LEARNED = 0, 1, 2, 3
MIX_FIXED, MIX_MORE, MIX_MORE_PRINTED = 0, 1, 2
XC_NONE, XC_LDA = 0, 1
TERM_NAMES = ("F_TF", "K_e", "F_vW", "E_H", "F_xc", "E_ie", "U_ii", "U_pp", "U_pm", "U_je", "alpha")
PTERM_NAMES = ("P_TF", "P_vW", "P_H", "P_xc", "P_ie", "P_ii")
STRESS_TERMS = ("i", "TF", "vW", "xc", "ee", "ie", "ii")  # ARCHE_S_* order
PROF_NAMES = ("scf_active", "fft_z", "fft_strided")
DBG = dict(Vie=0, Vi=1, n_a=2, n_i=3, SZ_plus=4, SZ_minus=5, nhat_a=6, F_pp=7)

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)


class ArcheError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("arche status %d: %s" % (status, msg))
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [
        ("n_atoms", ctypes.c_int32), ("n_species", ctypes.c_int32),
        ("species", _ip), ("Z", _dp), ("rc", _dp), ("mass", _dp),
        ("cell", ctypes.c_double * 3), ("grid", ctypes.c_int32 * 3),
        ("kT", ctypes.c_double), ("lambda_vw", ctypes.c_double), ("xc", ctypes.c_int32),
        ("scf_tol", ctypes.c_double), ("scf_max_iter", ctypes.c_int32), ("mixing", ctypes.c_int32),
        ("more_warmup", ctypes.c_int32), ("more_trust", ctypes.c_double), ("w_fixed", ctypes.c_double),
        ("init", ctypes.c_int32),
        ("ff_table", _dp), ("ff_len", ctypes.c_int32), ("ff_dq", ctypes.c_double),
        ("ewald_alpha", ctypes.c_double), ("exclusive_device", ctypes.c_int32),
    ]


class Result(ctypes.Structure):
    _fields_ = [
        ("F", ctypes.c_double), ("E", ctypes.c_double), ("terms", ctypes.c_double * 11),
        ("P", ctypes.c_double), ("pterms", ctypes.c_double * 6), ("mu", ctypes.c_double),
        ("residual", ctypes.c_double), ("w_last", ctypes.c_double),
        ("scf_iters", ctypes.c_int32), ("newton_iters", ctypes.c_int32),
        ("used_fallback", ctypes.c_int32), ("converged", ctypes.c_int32),
    ]

    def as_dict(self):
        return dict(F=self.F, E=self.E, terms=dict(zip(TERM_NAMES, list(self.terms))), P=self.P,
                    P_terms=dict(zip(PTERM_NAMES, list(self.pterms))), mu=self.mu, residual=self.residual,
                    w_last=self.w_last, scf_iters=self.scf_iters, newton_iters=self.newton_iters,
                    used_fallback=bool(self.used_fallback), converged=bool(self.converged))


class AAParams(ctypes.Structure):
    _fields_ = [("Z", ctypes.c_double), ("rho_ion", ctypes.c_double), ("kT", ctypes.c_double),
                ("r_cut_frac", ctypes.c_double), ("xc", ctypes.c_int32), ("n_radial", ctypes.c_int32)]


class AAResult(ctypes.Structure):
    _fields_ = [("r_ws", ctypes.c_double), ("r_cut", ctypes.c_double), ("mu", ctypes.c_double),
                ("dE_AA", ctypes.c_double), ("a", ctypes.c_double), ("b", ctypes.c_double), ("c", ctypes.c_double),
                ("iters", ctypes.c_int32)]


def aa_pseudopotential(Z, rho_ion, kT, r_cut_frac, xc=True, dq=0.01, n_q=400, n_radial=2001):
    """arche_aa_pseudopotential: (form-factor table D(i dq), result dict) of the
    average-atom pseudopotential (Sec. 2.4); the table goes to Options.ff_table."""
    p = AAParams(float(Z), float(rho_ion), float(kT), float(r_cut_frac), XC_LDA if xc else XC_NONE, int(n_radial))
    table = np.empty(int(n_q))
    r = AAResult()
    s = load().arche_aa_pseudopotential(ctypes.byref(p), float(dq), int(n_q), _ptr(table), ctypes.byref(r))
    if s != OK:
        raise ArcheError(s, "arche_aa_pseudopotential")
    return table, {k: getattr(r, k) for k, _ in AAResult._fields_}


class EosStat(ctypes.Structure):
    _fields_ = [("mean", ctypes.c_double), ("std", ctypes.c_double), ("sem", ctypes.c_double),
                ("tau", ctypes.c_double), ("n_used", ctypes.c_int64), ("n_eff", ctypes.c_int64),
                ("stride", ctypes.c_int64), ("start", ctypes.c_int64)]


def eos_average(series, thermal_fraction=0.2):
    """arche_eos_average: time average after the thermalisation cut, with the
    standard error from uncorrelated values (Sec. 4)."""
    x = _f64(series).reshape(-1)
    st = EosStat()
    s = load().arche_eos_average(_ptr(x), x.size, float(thermal_fraction), ctypes.byref(st))
    if s != OK:
        raise ArcheError(s, "arche_eos_average")
    return {k: getattr(st, k) for k, _ in EosStat._fields_}


_lib = None
_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_RELEASE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
_allocator_keep = None  # the installed callbacks (kept alive while installed)


def use_torch_allocator(on: bool = True):
    """Install (on=True) or remove PyTorch's caching allocator as the source of
    the device memory of contexts and batches created afterwards
    (arche_set_allocator).  Memory is requested on the context's stream and
    returned when the context is freed."""
    global _allocator_keep
    import torch
    L = load()
    if not on:
        s = L.arche_set_allocator(_ALLOC_FN(), _RELEASE_FN())
        if s != OK:
            raise ArcheError(s, "arche_set_allocator")
        _allocator_keep = None
        return

    def alloc(nbytes, stream):
        try:
            return int(torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0)))
        except Exception:
            return None

    def release(ptr, stream):
        torch.cuda.caching_allocator_delete(int(ptr))

    fa, fr = _ALLOC_FN(alloc), _RELEASE_FN(release)
    s = L.arche_set_allocator(fa, fr)
    if s != OK:
        raise ArcheError(s, "arche_set_allocator")
    _allocator_keep = (fa, fr)


def load(path: str = LIB_PATH):
    """Load libarche.so.  Raises if it has not been built: there is no fallback."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libarche.so not found at %s; run paper_2606_13283_amd.build.build()" % path)
    L = ctypes.CDLL(path)
    st = ctypes.c_int
    vp = ctypes.c_void_p
    L.arche_scf_init.argtypes = [ctypes.POINTER(Params), vp, ctypes.POINTER(vp)]
    L.arche_scf_init.restype = st
    L.arche_scf_solve.argtypes = [vp, _dp, ctypes.POINTER(Result)]
    L.arche_scf_solve.restype = st
    L.arche_forces.argtypes = [vp, _dp]
    L.arche_forces.restype = st
    L.arche_md_step.argtypes = [vp, ctypes.c_double, _dp, _dp, _dp, ctypes.POINTER(Result)]
    L.arche_md_step.restype = st
    L.arche_aa_pseudopotential.argtypes = [ctypes.POINTER(AAParams), ctypes.c_double, ctypes.c_int32, _dp,
                                            ctypes.POINTER(AAResult)]
    L.arche_aa_pseudopotential.restype = st
    L.arche_eos_average.argtypes = [_dp, ctypes.c_int64, ctypes.c_double, ctypes.POINTER(EosStat)]
    L.arche_eos_average.restype = st
    L.arche_md_predict.argtypes = [vp, ctypes.c_double, _dp, _dp, _dp]
    L.arche_md_predict.restype = st
    L.arche_learned_guide.argtypes = [vp, _dp, _dp]
    L.arche_learned_guide.restype = st
    L.arche_stress.argtypes = [vp, _dp, _dp, _dp]
    L.arche_stress.restype = st
    L.arche_get_density.argtypes = [vp, _dp, ctypes.c_int32]
    L.arche_get_density.restype = st
    L.arche_set_density.argtypes = [vp, _dp, ctypes.c_int32]
    L.arche_set_density.restype = st
    L.arche_reset_history.argtypes = [vp]
    L.arche_reset_history.restype = st
    L.arche_scf_free.argtypes = [vp]
    L.arche_scf_free.restype = None
    L.arche_last_error.argtypes = [vp]
    L.arche_last_error.restype = ctypes.c_char_p
    L.arche_version.argtypes = []
    L.arche_version.restype = ctypes.c_char_p
    L.arche_debug_get.argtypes = [vp, ctypes.c_int32, _dp]
    L.arche_debug_get.restype = st
    L.arche_debug_one_center.argtypes = [vp, _dp, _dp, _ip]
    L.arche_debug_one_center.restype = st
    L.arche_debug_one_center2.argtypes = [vp, _dp, _dp, _ip, _dp]
    L.arche_debug_one_center2.restype = st
    L.arche_profile_enable.argtypes = [vp, ctypes.c_int32]
    L.arche_profile_enable.restype = st
    L.arche_profile_reset.argtypes = [vp]
    L.arche_profile_sample.argtypes = [vp, ctypes.c_int32]
    L.arche_profile_sample.restype = st
    L.arche_profile_reset.restype = st
    L.arche_profile_read.argtypes = [vp, ctypes.c_int32, _dp, ctypes.POINTER(ctypes.c_int64)]
    L.arche_profile_read.restype = st
    L.arche_batch_init.argtypes = [ctypes.c_int32, ctypes.POINTER(Params), vp, ctypes.POINTER(vp)]
    L.arche_batch_init.restype = st
    L.arche_batch_solve.argtypes = [vp, ctypes.POINTER(_dp), ctypes.POINTER(Result), ctypes.POINTER(_dp)]
    L.arche_batch_solve.restype = st
    L.arche_batch_context.argtypes = [vp, ctypes.c_int32]
    L.arche_batch_context.restype = vp
    L.arche_batch_info.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    L.arche_batch_info.restype = st
    L.arche_batch_set_schedule.argtypes = [vp, ctypes.c_int32, ctypes.c_int32]
    L.arche_batch_set_schedule.restype = st
    L.arche_batch_last_error.argtypes = [vp]
    L.arche_batch_last_error.restype = ctypes.c_char_p
    L.arche_batch_free.argtypes = [vp]
    L.arche_batch_free.restype = None
    L.arche_scf_solve_batch.argtypes = [ctypes.c_int32, ctypes.POINTER(Params), ctypes.POINTER(_dp),
                                        ctypes.POINTER(Result), vp]
    L.arche_scf_solve_batch.restype = st
    L.arche_net_param_count.argtypes = []
    L.arche_net_param_count.restype = ctypes.c_int64
    L.arche_net_create.argtypes = [_ip, vp, ctypes.POINTER(vp)]
    L.arche_net_create.restype = st
    _fp = ctypes.POINTER(ctypes.c_float)
    for nm in ("arche_net_set_params", "arche_net_get_params", "arche_net_get_grads"):
        getattr(L, nm).argtypes = [vp, _fp, ctypes.c_int64]
        getattr(L, nm).restype = st
    L.arche_net_forward.argtypes = [vp, vp, vp, ctypes.c_double, vp]
    L.arche_net_forward.restype = st
    L.arche_net_propose.argtypes = [vp, vp, vp, ctypes.c_double, vp]
    L.arche_net_propose.restype = st
    L.arche_net_loss_grad.argtypes = [vp, vp, vp, vp, ctypes.c_double, _dp]
    L.arche_net_loss_grad.restype = st
    L.arche_net_adam_step.argtypes = [vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double]
    L.arche_net_adam_step.restype = st
    L.arche_net_debug_get.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, _fp]
    L.arche_net_debug_get.restype = st
    L.arche_net_sync.argtypes = [vp]
    L.arche_net_sync.restype = st
    L.arche_net_last_error.argtypes = [vp]
    L.arche_net_last_error.restype = ctypes.c_char_p
    L.arche_net_free.argtypes = [vp]
    L.arche_net_free.restype = None
    L.arche_set_init_net.argtypes = [vp, vp]
    L.arche_set_init_net.restype = st
    L.arche_debug_history.argtypes = [vp, _dp, ctypes.c_int32, _ip]
    L.arche_debug_history.restype = st
    L.arche_debug_live_contexts.argtypes = []
    L.arche_debug_live_contexts.restype = ctypes.c_int32
    L.arche_fft_tile.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    L.arche_fft_tile.restype = ctypes.c_int32
    L.arche_k_fft_r2c.argtypes = [_ip, vp, vp, vp]
    L.arche_k_fft_r2c.restype = st
    L.arche_k_fft_c2r.argtypes = [_ip, vp, vp, vp]
    L.arche_k_fft_c2r.restype = st
    L.arche_set_allocator.argtypes = [_ALLOC_FN, _RELEASE_FN]
    L.arche_set_allocator.restype = st
    L.arche_k_fft_c2r_noalloc.argtypes = [_ip, vp, vp, vp]
    L.arche_k_fft_c2r_noalloc.restype = st
    L.arche_k_fermi_dirac.argtypes = [ctypes.c_int64, vp, vp, vp, vp, vp]
    L.arche_k_fermi_dirac.restype = st
    L.arche_k_fermi_dirac_derivs.argtypes = [ctypes.c_int64, vp, vp, vp, vp, vp, vp]
    L.arche_k_fermi_dirac_derivs.restype = st
    _lib = L
    return L


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


def _ptr(a):
    return a.ctypes.data_as(_dp)


@dataclass
class Options:
    scf_tol: float = 1e-10
    scf_max_iter: int = 5000
    mixing: int = MIX_MORE
    more_warmup: int = 3
    more_trust: float = 0.5
    w_fixed: float = 0.95
    init: int = INIT_ONE_CENTER
    lambda_vw: float = 0.2
    xc: int = XC_LDA
    # tabulated non-Coulomb form factor D_s(q) = V_s(q) + Z_s/(pi q^2) at q = i ff_dq,
    # shape (n_species, ff_len); None: the analytic empty core of rc
    ff_table: object = None
    ff_dq: float = 0.0
    ewald_alpha: float = 0.0  # <= 0: automatic
    exclusive_device: int = 0  # 1: nothing else runs on the GPU (plain launch of the SCF kernel)


def _make_params(cell, grid, species, Z, rc, mass, kT, opts: Options | None = None):
    """arche_params for one system; returns it with the arrays it points to."""
    o = opts or Options()
    species = np.ascontiguousarray(np.asarray(species, dtype=np.int32).reshape(-1))
    Z, rc, mass = _f64(Z).reshape(-1), _f64(rc).reshape(-1), _f64(mass).reshape(-1)
    p = Params()
    p.n_atoms = species.size
    p.n_species = Z.size
    p.species = species.ctypes.data_as(_ip)
    p.Z, p.rc, p.mass = _ptr(Z), _ptr(rc), _ptr(mass)
    for a in range(3):
        p.cell[a] = float(cell[a])
        p.grid[a] = int(grid[a])
    p.kT = float(kT)
    p.lambda_vw = float(o.lambda_vw)
    p.xc = int(o.xc)
    p.scf_tol = float(o.scf_tol)
    p.scf_max_iter = int(o.scf_max_iter)
    p.mixing = int(o.mixing)
    p.more_warmup = int(o.more_warmup)
    p.more_trust = float(o.more_trust)
    p.w_fixed = float(o.w_fixed)
    p.init = int(o.init)
    keep = [species, Z, rc, mass]
    if o.ff_table is not None:
        ff = np.ascontiguousarray(np.asarray(o.ff_table, dtype=np.float64).reshape(Z.size, -1))
        keep.append(ff)
        p.ff_table = _ptr(ff)
        p.ff_len = ff.shape[1]
        p.ff_dq = float(o.ff_dq)
    p.ewald_alpha = float(o.ewald_alpha)
    p.exclusive_device = int(o.exclusive_device)
    return p, tuple(keep)


class Context:
    """One system (cell, grid, species, temperature) on the current HIP device."""

    def __init__(self, cell, grid, species, Z, rc, mass, kT, opts: Options | None = None, stream=None):
        L = load()
        p, keep = _make_params(cell, grid, species, Z, rc, mass, kT, opts)
        h = ctypes.c_void_p()
        s = L.arche_scf_init(ctypes.byref(p), ctypes.c_void_p(stream) if stream else None, ctypes.byref(h))
        if s != OK:
            raise ArcheError(s, L.arche_last_error(None).decode())
        self._setup(L, h, p, keep, owned=True)

    def _setup(self, L, h, p, keep, owned):
        self._keep = keep
        self.params = p
        self.n_atoms = p.n_atoms
        self.grid = tuple(int(p.grid[a]) for a in range(3))
        self.nh = self.grid[0] * self.grid[1] * (self.grid[2] // 2 + 1)
        self._h = h
        self._L = L
        self._owned = owned

    @classmethod
    def from_workload(cls, w, opts: Options | None = None, stream=None):
        return cls(w.cell, w.grid, w.species, w.Z, w.rc, w.mass, w.kT, opts, stream)

    def _check(self, s, allow=()):
        if s != OK and s not in allow:
            raise ArcheError(s, self._L.arche_last_error(self._h).decode())
        return s

    def solve(self, pos, allow_noconv=False):
        pos = _f64(pos, (self.n_atoms, 3))
        r = Result()
        s = self._L.arche_scf_solve(self._h, _ptr(pos), ctypes.byref(r))
        self._check(s, (ENOCONV,) if allow_noconv else ())
        return r.as_dict()

    def forces(self):
        F = np.empty((self.n_atoms, 3))
        self._check(self._L.arche_forces(self._h, _ptr(F)))
        return F

    def md_step(self, dt, pos, vel):
        pos = _f64(pos, (self.n_atoms, 3)).copy()
        vel = _f64(vel, (self.n_atoms, 3)).copy()
        F = np.empty((self.n_atoms, 3))
        r = Result()
        self._check(self._L.arche_md_step(self._h, float(dt), _ptr(pos), _ptr(vel), _ptr(F), ctypes.byref(r)))
        return pos, vel, F, r.as_dict()

    def md_predict(self, dt, pos, vel):
        """r(t+dt) that md_step would move to (no solve)."""
        pos = _f64(pos, (self.n_atoms, 3))
        vel = _f64(vel, (self.n_atoms, 3))
        out = np.empty((self.n_atoms, 3))
        self._check(self._L.arche_md_predict(self._h, float(dt), _ptr(pos), _ptr(vel), _ptr(out)))
        return out

    def learned_guide(self, next_pos):
        """The learned proposal's guide G at the next positions (arche_learned_guide)."""
        next_pos = _f64(next_pos, (self.n_atoms, 3))
        out = np.empty(self.grid)
        self._check(self._L.arche_learned_guide(self._h, _ptr(next_pos), _ptr(out)))
        return out

    def stress(self, vel=None):
        """(total 3x3 stress tensor, {term: 3x3}) at the last converged solve (Sec. 2.6)."""
        sig = np.empty((3, 3))
        terms = np.empty((len(STRESS_TERMS), 3, 3))
        v = None if vel is None else _f64(vel, (self.n_atoms, 3))
        self._check(self._L.arche_stress(self._h, None if v is None else _ptr(v), _ptr(sig), _ptr(terms)))
        return sig, dict(zip(STRESS_TERMS, terms))

    def density(self):
        n = np.empty(self.grid)
        self._check(self._L.arche_get_density(self._h, _ptr(n), 0))
        return n

    def set_density(self, n):
        n = _f64(n, self.grid)
        self._check(self._L.arche_set_density(self._h, _ptr(n), 0))

    def set_init_net(self, net):
        """Use `net` (a Net on the same grid, or None) for INIT_LEARNED solves."""
        self._net = net
        self._check(self._L.arche_set_init_net(self._h, net._h if net is not None else None))

    def reset_history(self):
        self._check(self._L.arche_reset_history(self._h))

    def debug(self, name):
        w = DBG[name]
        if name in ("SZ_plus", "SZ_minus", "nhat_a"):
            out = np.empty(2 * self.nh)
            self._check(self._L.arche_debug_get(self._h, w, _ptr(out)))
            return out.view(np.complex128).reshape(self.grid[0], self.grid[1], self.grid[2] // 2 + 1)
        if name == "F_pp":
            out = np.empty((self.n_atoms, 3))
        else:
            out = np.empty(self.grid)
        self._check(self._L.arche_debug_get(self._h, w, _ptr(out)))
        return out

    def history(self):
        """Per-iteration rows of the last solve: iteration, residual, w, mu, K, U,
        max |dn|/n_a, Newton passes, More on, error."""
        n = ctypes.c_int32(0)
        self._check(self._L.arche_debug_history(self._h, None, 0, ctypes.byref(n)))
        out = np.zeros((n.value, 10))
        if n.value:
            self._check(self._L.arche_debug_history(self._h, _ptr(out), n.value, ctypes.byref(n)))
        return out

    def one_center_guess(self, pos):
        pos = _f64(pos, (self.n_atoms, 3))
        out = np.empty(self.grid)
        fb = ctypes.c_int32(0)
        self._check(self._L.arche_debug_one_center(self._h, _ptr(pos), _ptr(out), ctypes.byref(fb)))
        return out, bool(fb.value)

    def one_center_raw(self, pos):
        """(plain guess, used_fallback, guide G of the learned proposal) at pos."""
        pos = _f64(pos, (self.n_atoms, 3))
        out = np.empty(self.grid)
        raw = np.empty(self.grid)
        fb = ctypes.c_int32(0)
        self._check(self._L.arche_debug_one_center2(self._h, _ptr(pos), _ptr(out), ctypes.byref(fb), _ptr(raw)))
        return out, bool(fb.value), raw

    def profile(self, on=True, kinds=None):
        """Per-kernel event timing; kinds: names from PROF_NAMES (default all)."""
        if not on:
            code = 0
        elif kinds is None:
            code = 1
        else:
            code = sum(2 << PROF_NAMES.index(k) for k in kinds)
        self._check(self._L.arche_profile_enable(self._h, code))

    def profile_sample(self, every):
        """Time one launch in `every` of each kind."""
        self._check(self._L.arche_profile_sample(self._h, int(every)))

    def profile_reset(self):
        self._check(self._L.arche_profile_reset(self._h))

    def profile_read(self):
        out = {}
        for k, name in enumerate(PROF_NAMES):
            ms = ctypes.c_double(0.0)
            n = ctypes.c_int64(0)
            self._check(self._L.arche_profile_read(self._h, k, ctypes.byref(ms), ctypes.byref(n)))
            out[name] = (ms.value, n.value)
        return out

    def close(self):
        if getattr(self, "_h", None):
            if self._owned:
                self._L.arche_scf_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent systems solved together (arche_batch_*): one launch per
    pass over all unconverged snapshots, graph-captured iterations, results
    bit-identical to Context.solve on the same system."""

    def __init__(self, systems, stream=None):
        """systems: list of (cell, grid, species, Z, rc, mass, kT, Options)."""
        L = load()
        self._L = L
        made = [_make_params(*sy) for sy in systems]
        self._keep = [k for _, k in made]
        self.params = [p for p, _ in made]
        arr = (Params * len(made))(*self.params)
        self._arr = arr
        self.n = len(made)
        self.n_atoms = [p.n_atoms for p in self.params]
        h = ctypes.c_void_p()
        s = L.arche_batch_init(self.n, arr, ctypes.c_void_p(stream) if stream else None, ctypes.byref(h))
        if s != OK:
            raise ArcheError(s, "arche_batch_init failed")
        self._h = h

    @classmethod
    def from_workloads(cls, ws, opts_of=None, stream=None):
        opts_of = opts_of or (lambda w: Options(w_fixed=w.w_fixed, lambda_vw=w.lam,
                                                xc=XC_LDA if w.xc else XC_NONE, init=INIT_UNIFORM))
        return cls([(w.cell, w.grid, w.species, w.Z, w.rc, w.mass, w.kT, opts_of(w)) for w in ws], stream)

    def _check(self, s, allow=()):
        if s != OK and s not in allow:
            raise ArcheError(s, self._L.arche_batch_last_error(self._h).decode())
        return s

    def solve(self, positions, forces=False, allow_noconv=False):
        """Returns the result dicts (and the force arrays when forces=True)."""
        pos = [_f64(p, (n, 3)) for p, n in zip(positions, self.n_atoms)]
        pp = (_dp * self.n)(*[_ptr(p) for p in pos])
        res = (Result * self.n)()
        F = [np.empty((n, 3)) for n in self.n_atoms] if forces else None
        fp = (_dp * self.n)(*[_ptr(f) for f in F]) if forces else None
        s = self._L.arche_batch_solve(self._h, pp, res, fp)
        self._check(s, (ENOCONV,) if allow_noconv else ())
        out = [r.as_dict() for r in res]
        return (out, F) if forces else out

    def context(self, i):
        """Non-owning Context for snapshot i (density, debug, single solves)."""
        h = self._L.arche_batch_context(self._h, int(i))
        if not h:
            raise IndexError(i)
        c = Context.__new__(Context)
        c._setup(self._L, ctypes.c_void_p(h), self.params[i], self._keep[i], owned=False)
        return c

    def info(self):
        a = (ctypes.c_int32 * 6)()
        self._check(self._L.arche_batch_info(self._h, a))
        return {"coop_blocks": a[0], "iters_per_graph": a[1], "graph_whole_iteration": bool(a[2]),
                "graph_launches": a[3], "compactions": a[4], "tuned_now": bool(a[5])}

    def set_schedule(self, coop_blocks=0, iters_per_graph=0):
        self._check(self._L.arche_batch_set_schedule(self._h, int(coop_blocks), int(iters_per_graph)))

    def close(self):
        if getattr(self, "_h", None):
            self._L.arche_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Net:
    """The learned initial-density U-Net (arche_net_*).  Fields are FP64 torch
    tensors on the HIP device (torch supplies the memory only); parameters are
    FP32 numpy arrays in the documented order."""

    def __init__(self, grid, stream=None):
        L = load()
        self._L = L
        self.grid = tuple(int(g) for g in grid)
        g = (ctypes.c_int32 * 3)(*self.grid)
        h = ctypes.c_void_p()
        s = L.arche_net_create(g, ctypes.c_void_p(stream) if stream else None, ctypes.byref(h))
        if s != OK:
            raise ArcheError(s, "arche_net_create failed (grid edges multiples of 8, product of 16384)")
        self._h = h
        self.n_params = int(L.arche_net_param_count())

    def _check(self, s):
        if s != OK:
            raise ArcheError(s, self._L.arche_net_last_error(self._h).decode())

    @staticmethod
    def _dev(t):
        assert t.is_cuda and t.dtype.is_floating_point and t.is_contiguous()
        return ctypes.c_void_p(t.data_ptr())

    def set_params(self, p):
        p = np.ascontiguousarray(np.asarray(p, dtype=np.float32).reshape(-1))
        self._check(self._L.arche_net_set_params(self._h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), p.size))

    def params(self):
        p = np.empty(self.n_params, dtype=np.float32)
        self._check(self._L.arche_net_get_params(self._h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), p.size))
        return p

    def grads(self):
        p = np.empty(self.n_params, dtype=np.float32)
        self._check(self._L.arche_net_get_grads(self._h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), p.size))
        return p

    def forward(self, guess, prev, n0, r_out):
        self._check(self._L.arche_net_forward(self._h, self._dev(guess), self._dev(prev), float(n0), self._dev(r_out)))

    def propose(self, guess, prev, n0, n_out):
        self._check(self._L.arche_net_propose(self._h, self._dev(guess), self._dev(prev), float(n0), self._dev(n_out)))

    def loss_grad(self, guess, prev, conv, n0):
        loss = ctypes.c_double(0.0)
        self._check(self._L.arche_net_loss_grad(self._h, self._dev(guess), self._dev(prev), self._dev(conv),
                                                float(n0), ctypes.byref(loss)))
        return loss.value

    def adam_step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self._check(self._L.arche_net_adam_step(self._h, float(lr), float(beta1), float(beta2), float(eps)))

    def debug(self, which, level):
        g = [x >> level for x in self.grid]
        out = np.empty((g[0], g[1], g[2], 32), dtype=np.float32)
        self._check(self._L.arche_net_debug_get(self._h, int(which), int(level),
                                                out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return out

    def sync(self):
        self._check(self._L.arche_net_sync(self._h))

    def close(self):
        if getattr(self, "_h", None):
            self._L.arche_net_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- kernel-level calls on torch device tensors ----

def _grid_arr(grid):
    return (ctypes.c_int32 * 3)(*[int(g) for g in grid])


def fft_r2c(x):
    """Unnormalised rfftn of a contiguous float64 cuda tensor [Nx, Ny, Nz] -> complex128 tensor."""
    import torch
    L = load()
    x = x.contiguous()
    Nx, Ny, Nz = x.shape
    out = torch.empty((Nx, Ny, Nz // 2 + 1), dtype=torch.complex128, device=x.device)
    s = L.arche_k_fft_r2c(_grid_arr(x.shape), ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                          ctypes.c_void_p(torch.cuda.current_stream(x.device).cuda_stream))
    if s != OK:
        raise ArcheError(s, "arche_k_fft_r2c")
    return out


def fft_c2r(X, Nz):
    """Unnormalised inverse of fft_r2c (numpy irfftn times N) for a complex128 cuda tensor."""
    import torch
    L = load()
    X = X.contiguous()
    Nx, Ny, _ = X.shape
    out = torch.empty((Nx, Ny, Nz), dtype=torch.float64, device=X.device)
    s = L.arche_k_fft_c2r(_grid_arr((Nx, Ny, Nz)), ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                          ctypes.c_void_p(torch.cuda.current_stream(X.device).cuda_stream))
    if s != OK:
        raise ArcheError(s, "arche_k_fft_c2r")
    return out


NOALLOC_MAX_NH = 1064960  # ARCHE_NOALLOC_MAX_NH


def fft_c2r_noalloc(X, Nz, out=None):
    """fft_c2r through the allocation-free entry point, into `out` (allocated here
    when None, so that callers that cannot allocate pass their own).  Enqueued on
    torch's current stream; not synchronised."""
    import torch
    L = load()
    X = X.contiguous()
    Nx, Ny, _ = X.shape
    if out is None:
        out = torch.empty((Nx, Ny, Nz), dtype=torch.float64, device=X.device)
    s = L.arche_k_fft_c2r_noalloc(_grid_arr((Nx, Ny, Nz)), ctypes.c_void_p(X.data_ptr()),
                                  ctypes.c_void_p(out.data_ptr()),
                                  ctypes.c_void_p(torch.cuda.current_stream(X.device).cuda_stream))
    if s != OK:
        raise ArcheError(s, "arche_k_fft_c2r_noalloc")
    return out


def fermi_dirac(x):
    """(I_{-1/2}, I_{1/2}, I_{3/2}) of a float64 cuda tensor."""
    import torch
    L = load()
    x = x.contiguous()
    a, b, c = (torch.empty_like(x) for _ in range(3))
    s = L.arche_k_fermi_dirac(x.numel(), ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(a.data_ptr()),
                              ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(c.data_ptr()),
                              ctypes.c_void_p(torch.cuda.current_stream(x.device).cuda_stream))
    if s != OK:
        raise ArcheError(s, "arche_k_fermi_dirac")
    return a, b, c


def fermi_dirac_derivs(x):
    """I_{1/2} and its first three derivatives at a float64 cuda tensor, from the SCF kernel's table."""
    import torch
    L = load()
    x = x.contiguous()
    out = [torch.empty_like(x) for _ in range(4)]
    s = L.arche_k_fermi_dirac_derivs(x.numel(), ctypes.c_void_p(x.data_ptr()),
                                     *[ctypes.c_void_p(o.data_ptr()) for o in out],
                                     ctypes.c_void_p(torch.cuda.current_stream(x.device).cuda_stream))
    if s != OK:
        raise ArcheError(s, "arche_k_fermi_dirac_derivs")
    return tuple(out)


def version():
    return load().arche_version().decode()
