"""ctypes binding of libebit.so (argument marshalling only).

Every step of the path runs in the HIP library.  Device memory and the
stream come from PyTorch: tensors must be CUDA (HIP) tensors, contiguous, of
the dtype each call documents.  If the library has not been built, loading
raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libebit.so")

OK, EINVAL, ENOMEM, EGEOM, ENOCONV, ENAN, EHIP, ESTATE, EIO = 0, -1, -2, -3, -4, -5, -6, -7, -8
FP64, MIXED = 0, 1
OUTER_PCG, OUTER_DC = 0, 1
SYS_HEAT, SYS_PRESSURE = 0, 1
NEUMANN, DIRICHLET, PERIODIC = 0, 1, 2


class Grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int * 3), ("h", ctypes.c_double),
                ("T_bc", ctypes.c_int * 6), ("T_val", ctypes.c_double * 6),
                ("p_bc", ctypes.c_int * 6), ("p_val", ctypes.c_double * 6)]


class Props(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in ("rho_l", "rho_v", "lam_l", "lam_v", "cp_l", "cp_v", "h_lg", "T_sat")]


class Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("outer", ctypes.c_int), ("rtol", ctypes.c_double),
                ("max_iters", ctypes.c_int), ("nu1", ctypes.c_int), ("nu2", ctypes.c_int),
                ("theta_min", ctypes.c_double), ("check_every", ctypes.c_int), ("tail_cells", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("vcycles", ctypes.c_int), ("rel_res", ctypes.c_double),
                ("bnorm", ctypes.c_double), ("res_floor", ctypes.c_double), ("seconds", ctypes.c_double),
                ("div_max", ctypes.c_double),
                ("fallbacks", ctypes.c_int), ("status", ctypes.c_int), ("fp64_fallback", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None
_P3 = ctypes.c_void_p * 3


def load():
    """Load libebit.so; raises if it is missing (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run `python __graft_entry__.py` (build()) first")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    sig = {
        "ebit_default_opts": (None, [ctypes.POINTER(Opts)]),
        "ebit_status_string": (ctypes.c_char_p, [i]),
        "ebit_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(Grid), ctypes.POINTER(Opts)]),
        "ebit_create": (i, [ctypes.POINTER(vp), ctypes.POINTER(Grid), ctypes.POINTER(Props), ctypes.POINTER(Opts),
                            vp, ctypes.c_size_t, vp]),
        "ebit_destroy": (i, [vp]),
        "ebit_last_error": (ctypes.c_char_p, [vp]),
        "ebit_build_coeffs": (i, [vp, _P3, vp, vp, d]),
        "ebit_heat_solve": (i, [vp, vp, vp, i, ctypes.POINTER(Stats)]),
        "ebit_mass_flux": (i, [vp, vp, vp, vp, ctypes.POINTER(Stats)]),
        "ebit_project": (i, [vp, _P3, _P3, vp, vp, i, ctypes.POINTER(Stats)]),
        "ebit_get_geometry": (i, [vp, vp, vp, vp]),
        "ebit_apply": (i, [vp, i, vp, vp]),
        "ebit_heat_rhs": (i, [vp, vp, vp]),
        "ebit_extend": (i, [vp, vp, i, i]),
        "ebit_ghost_band": (i, [vp, _P3, _P3, vp]),
        "ebit_volume_fraction": (i, [vp, _P3, vp, vp]),
        "ebit_project_one_fluid": (i, [vp, _P3, vp, vp, i, ctypes.POINTER(Stats)]),
        "ebit_project_rhs": (i, [vp, _P3, _P3, vp, vp]),
        "ebit_levels": (i, [vp, ctypes.POINTER(i), ctypes.POINTER(i)]),
        "ebit_profile": (i, [vp, i]),
        "ebit_profile_read": (i, [vp, i, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(d)]),
        "ebit_batch_workspace_bytes": (ctypes.c_size_t, [i, ctypes.POINTER(Opts)]),
        "ebit_batch_create": (i, [ctypes.POINTER(vp), i, ctypes.POINTER(vp), vp, ctypes.c_size_t, vp]),
        "ebit_batch_destroy": (i, [vp]),
        "ebit_batch_last_error": (ctypes.c_char_p, [vp]),
        "ebit_batch_build_coeffs": (i, [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                        ctypes.POINTER(d)]),
        "ebit_batch_heat_solve": (i, [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), i, ctypes.POINTER(Stats)]),
        "ebit_batch_mass_flux": (i, [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(Stats)]),
        "ebit_batch_project": (i, [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                   ctypes.POINTER(vp), i, ctypes.POINTER(Stats)]),
        "ebit_autotune": (i, [vp, vp, vp, vp, ctypes.POINTER(Opts), ctypes.POINTER(d)]),
        "ebit_batch_autotune": (i, [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                    ctypes.POINTER(Opts), ctypes.POINTER(d)]),
        "ebit_cut_fractions_noalloc": (i, [ctypes.POINTER(Grid), _P3, vp, vp, _P3, vp, vp]),
        "ebit_interface_velocity": (i, [vp, _P3, _P3, vp, _P3]),
        "ebit_advect_markers": (i, [vp, _P3, _P3, vp, vp, d]),
        "ebit_advect_energy": (i, [vp, vp, vp, _P3, _P3, vp, d, d, vp]),
        "ebit_tune_lookup": (i, [ctypes.c_char_p, ctypes.POINTER(Grid), ctypes.POINTER(Opts), ctypes.POINTER(Opts),
                                 ctypes.POINTER(i)]),
        "ebit_tune_store": (i, [ctypes.c_char_p, ctypes.POINTER(Grid), ctypes.POINTER(Opts), d]),
        "ebit_autotune_cached": (i, [vp, ctypes.c_char_p, vp, vp, vp, ctypes.POINTER(Opts), ctypes.POINTER(d),
                                     ctypes.POINTER(i)]),
        "ebit_batch_autotune_cached": (i, [vp, ctypes.c_char_p, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                           ctypes.POINTER(vp), ctypes.POINTER(Opts), ctypes.POINTER(d),
                                           ctypes.POINTER(i)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


EXPORTED = ["ebit_default_opts", "ebit_status_string", "ebit_workspace_bytes", "ebit_create", "ebit_destroy",
            "ebit_last_error", "ebit_build_coeffs", "ebit_heat_solve", "ebit_mass_flux", "ebit_project",
            "ebit_get_geometry", "ebit_apply", "ebit_heat_rhs", "ebit_extend", "ebit_project_one_fluid", "ebit_project_rhs", "ebit_levels",
            "ebit_profile", "ebit_profile_read", "ebit_batch_workspace_bytes", "ebit_batch_create",
            "ebit_batch_destroy", "ebit_batch_last_error", "ebit_batch_build_coeffs", "ebit_batch_heat_solve",
            "ebit_batch_mass_flux", "ebit_batch_project", "ebit_autotune", "ebit_batch_autotune",
            "ebit_cut_fractions_noalloc", "ebit_interface_velocity", "ebit_advect_markers", "ebit_advect_energy",
            "ebit_tune_lookup", "ebit_tune_store", "ebit_autotune_cached", "ebit_batch_autotune_cached",
            "ebit_ghost_band", "ebit_volume_fraction"]
NOALLOC_MAX_CELLS = 1 << 18
KC_FINE_SMOOTH, KC_FINE_RESTRICT, KC_COARSE, KC_OUTER_APPLY, KC_OUTER_UPDATE, KC_TAIL = range(6)
EXT_LIQ_TO_VAP, EXT_VAP_TO_LIQ, EXT_IFACE_TO_BAND = range(3)


class EbitError(RuntimeError):
    def __init__(self, status, where, detail=""):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} ({status}) {detail}")


def status_string(s):
    return load().ebit_status_string(int(s)).decode()


def default_opts(**kw) -> Opts:
    o = Opts()
    load().ebit_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def make_grid(dim, n, h, T_bc, p_bc) -> Grid:
    g = Grid()
    g.dim = dim
    for a in range(3):
        g.n[a] = int(n[a])
    g.h = float(h)
    for s in range(6):
        kT, vT = T_bc[s] if s < len(T_bc) else (0, 0.0)
        kp, vp = p_bc[s] if s < len(p_bc) else (0, 0.0)
        g.T_bc[s], g.T_val[s] = int(kT), float(vT)
        g.p_bc[s], g.p_val[s] = int(kp), float(vp)
    return g


def make_props(p) -> Props:
    q = Props()
    for k, _ in Props._fields_:
        setattr(q, k, float(getattr(p, k)))
    return q


def _ptr(t: Optional[torch.Tensor], dtype=None):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    return ctypes.c_void_p(t.data_ptr())


def _p3(ts: Optional[Sequence[torch.Tensor]], dtype=torch.float64):
    if ts is None:
        return None
    arr = _P3()
    for a in range(3):
        arr[a] = _ptr(ts[a], dtype).value if a < len(ts) and ts[a] is not None else None
    return arr


class Context:
    """One grid + properties + options; owns a torch-allocated workspace."""

    def __init__(self, grid: Grid, props: Props, opts: Optional[Opts] = None, device="cuda",
                 stream: Optional[torch.cuda.Stream] = None):
        lib = load()
        self.lib = lib
        self.grid, self.props = grid, props
        self.opts = opts if opts is not None else default_opts()
        nbytes = lib.ebit_workspace_bytes(ctypes.byref(grid), ctypes.byref(self.opts))
        if nbytes == 0:
            raise EbitError(EINVAL, "ebit_workspace_bytes", "(invalid grid)")
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        self.ws_bytes = nbytes
        h = ctypes.c_void_p()
        st = lib.ebit_create(ctypes.byref(h), ctypes.byref(grid), ctypes.byref(props), ctypes.byref(self.opts),
                             ctypes.c_void_p(aligned), ctypes.c_size_t(nbytes),
                             ctypes.c_void_p(self.stream.cuda_stream))
        if st != OK:
            raise EbitError(st, "ebit_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.ebit_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, where):
        if st != OK:
            raise EbitError(st, where, self.lib.ebit_last_error(self.h).decode())

    # -- entry points -------------------------------------------------------
    def build_coeffs(self, markers, vcol, ccol, dt):
        self._check(self.lib.ebit_build_coeffs(self.h, _p3(markers), _ptr(vcol, torch.uint8),
                                               _ptr(ccol, torch.uint8), float(dt)), "ebit_build_coeffs")

    def heat_solve(self, T_star, T, use_guess=False, check=True):
        s = Stats()
        st = self.lib.ebit_heat_solve(self.h, _ptr(T_star, torch.float64), _ptr(T, torch.float64),
                                      int(use_guess), ctypes.byref(s))
        if check:
            self._check(st, "ebit_heat_solve")
        return s.as_dict()

    def mass_flux(self, T, mdot, mdot_face=None, stats=True):
        """mdot from T; with stats=False the call does not wait for the
        device and returns None."""
        s = Stats()
        st = self.lib.ebit_mass_flux(self.h, _ptr(T, torch.float64), _ptr(mdot, torch.float64),
                                     _p3(mdot_face), ctypes.byref(s) if stats else None)
        self._check(st, "ebit_mass_flux")
        return s.as_dict() if stats else None

    def project(self, u_l, u_v, mdot, p, use_guess=False, check=True):
        s = Stats()
        st = self.lib.ebit_project(self.h, _p3(u_l), _p3(u_v), _ptr(mdot, torch.float64),
                                   _ptr(p, torch.float64), int(use_guess), ctypes.byref(s))
        if check:
            self._check(st, "ebit_project")
        return s.as_dict()

    def project_one_fluid(self, u, mdot, p, use_guess=False, check=True):
        """One-fluid projection (Eq. pc_source): u (dim face arrays, in
        place), mdot per cell, p output; returns the stats as a dict."""
        s = Stats()
        st = self.lib.ebit_project_one_fluid(self.h, _p3(u), _ptr(mdot, torch.float64), _ptr(p, torch.float64),
                                             int(use_guess), ctypes.byref(s))
        if check:
            self._check(st, "ebit_project_one_fluid")
        return s.as_dict()

    def get_geometry(self, theta=None, flags=None, facet=None):
        self._check(self.lib.ebit_get_geometry(self.h, _p3(theta), _ptr(flags, torch.uint8),
                                               _ptr(facet, torch.float64)), "ebit_get_geometry")

    def apply(self, system, x, y):
        self._check(self.lib.ebit_apply(self.h, int(system), _ptr(x, torch.float64), _ptr(y, torch.float64)),
                    "ebit_apply")

    def extend(self, q, mode, iters):
        """Eq. extrapolation: `iters` pseudo-time steps carrying q (cells,
        in place) into the narrow band; mode EXT_LIQ_TO_VAP, EXT_VAP_TO_LIQ
        or EXT_IFACE_TO_BAND."""
        self._check(self.lib.ebit_extend(self.h, _ptr(q, torch.float64), int(mode), int(iters)), "ebit_extend")

    def volume_fraction(self, markers, vcol, frac, check=True):
        """Liquid volume fraction of every cell (2D) into frac (cells) from
        the markers and vertex colours; returns the status."""
        st = self.lib.ebit_volume_fraction(self.h, _p3(markers), _ptr(vcol, torch.uint8), _ptr(frac, torch.float64))
        if check:
            self._check(st, "ebit_volume_fraction")
        return st

    def ghost_band(self, u_l, u_v, mdot_band, check=True):
        """Eq. ghost_velocity on every narrow-band face (u_l, u_v: dim face
        arrays, in place) from the band-extended mdot; returns the status."""
        st = self.lib.ebit_ghost_band(self.h, _p3(u_l), _p3(u_v), _ptr(mdot_band, torch.float64))
        if check:
            self._check(st, "ebit_ghost_band")
        return st

    def interface_velocity(self, u_l, u_v, mdot, u_gamma):
        """Eq. jump_interfacial_vel at the cell centres: u_gamma (dim cell
        arrays, written) from the face fields u_l, u_v and the
        band-extended mdot."""
        self._check(self.lib.ebit_interface_velocity(self.h, _p3(u_l), _p3(u_v), _ptr(mdot, torch.float64),
                                                     _p3(u_gamma)), "ebit_interface_velocity")

    def advect_markers(self, u_gamma, markers, vcol, ccol, dt, check=True):
        """One step of the EBIT markers (2D, x pass then y pass): markers,
        vcol and ccol in place; returns the status code."""
        st = self.lib.ebit_advect_markers(self.h, _p3(u_gamma), _p3(markers), _ptr(vcol, torch.uint8),
                                          _ptr(ccol, torch.uint8), float(dt))
        if check:
            self._check(st, "ebit_advect_markers")
        return st

    def advect_energy(self, T_liq, T_vap, u_l, u_v, ccol, dt, T_star, eps=1e-6, check=True):
        """Eq. energy_advection: T_star (cells, written) from each cell's
        own phase field (T_liq / T_vap, extended across the interface) and
        face velocities (u_l / u_v); returns the status code."""
        st = self.lib.ebit_advect_energy(self.h, _ptr(T_liq, torch.float64), _ptr(T_vap, torch.float64), _p3(u_l),
                                         _p3(u_v), _ptr(ccol, torch.uint8), float(dt), float(eps),
                                         _ptr(T_star, torch.float64))
        if check:
            self._check(st, "ebit_advect_energy")
        return st

    def heat_rhs(self, T_star, b):
        self._check(self.lib.ebit_heat_rhs(self.h, _ptr(T_star, torch.float64), _ptr(b, torch.float64)),
                    "ebit_heat_rhs")

    def project_rhs(self, u_l, u_v, mdot, b):
        self._check(self.lib.ebit_project_rhs(self.h, _p3(u_l), _p3(u_v), _ptr(mdot, torch.float64),
                                              _ptr(b, torch.float64)), "ebit_project_rhs")

    def profile(self, enable=True):
        self._check(self.lib.ebit_profile(self.h, int(enable)), "ebit_profile")

    def profile_read(self, kernel_class):
        n = ctypes.c_longlong()
        ms = ctypes.c_double()
        self._check(self.lib.ebit_profile_read(self.h, int(kernel_class), ctypes.byref(n), ctypes.byref(ms)),
                    "ebit_profile_read")
        return n.value, ms.value

    def autotune(self, b_heat=None, b_press=None, x=None):
        """Choose nu1 = nu2, tail_cells and check_every by timing solves of
        the given right-hand sides; returns (chosen options dict, ms)."""
        o = Opts()
        ms = ctypes.c_double()
        if x is None:
            x = torch.empty_like(b_heat if b_heat is not None else b_press)
        self._check(self.lib.ebit_autotune(self.h, _ptr(b_heat, torch.float64), _ptr(b_press, torch.float64),
                                           _ptr(x, torch.float64), ctypes.byref(o), ctypes.byref(ms)),
                    "ebit_autotune")
        self.opts = o
        return {k: getattr(o, k) for k, _ in Opts._fields_}, ms.value

    def autotune_cached(self, path, b_heat=None, b_press=None, x=None):
        """autotune through the schedule cache file at path; returns
        (chosen options dict, ms, from_cache)."""
        o = Opts()
        ms = ctypes.c_double()
        hit = ctypes.c_int()
        if x is None:
            x = torch.empty_like(b_heat if b_heat is not None else b_press)
        self._check(self.lib.ebit_autotune_cached(self.h, str(path).encode(), _ptr(b_heat, torch.float64),
                                                  _ptr(b_press, torch.float64), _ptr(x, torch.float64),
                                                  ctypes.byref(o), ctypes.byref(ms), ctypes.byref(hit)),
                    "ebit_autotune_cached")
        self.opts = o
        return {k: getattr(o, k) for k, _ in Opts._fields_}, ms.value, bool(hit.value)

    def levels(self):
        n = ctypes.c_int()
        sizes = (ctypes.c_int * (3 * 32))()
        self._check(self.lib.ebit_levels(self.h, ctypes.byref(n), sizes), "ebit_levels")
        return [tuple(sizes[3 * l: 3 * l + 3]) for l in range(n.value)]


def tune_lookup(path, grid, base):
    """ebit_tune_lookup (host only): (found, Opts) for the grid's key."""
    lib = load()
    out = Opts()
    found = ctypes.c_int()
    st = lib.ebit_tune_lookup(str(path).encode(), ctypes.byref(grid), ctypes.byref(base), ctypes.byref(out),
                              ctypes.byref(found))
    if st != OK:
        raise EbitError(st, "ebit_tune_lookup", "")
    return bool(found.value), out


def tune_store(path, grid, chosen, ms):
    """ebit_tune_store (host only); returns the status code."""
    return load().ebit_tune_store(str(path).encode(), ctypes.byref(grid), ctypes.byref(chosen), float(ms))


def cut_fractions_noalloc(grid, markers, vcol, ccol, theta, flags, stream=None):
    """ebit_cut_fractions_noalloc: theta (per-axis face arrays) and flags of
    the geometry pass with no context, workspace or allocation; returns the
    status code (0 = EBIT_OK)."""
    lib = load()
    st = stream if stream is not None else torch.cuda.current_stream()
    return lib.ebit_cut_fractions_noalloc(ctypes.byref(grid), _p3(markers), _ptr(vcol, torch.uint8),
                                          _ptr(ccol, torch.uint8), _p3(theta), _ptr(flags, torch.uint8),
                                          ctypes.c_void_p(st.cuda_stream))


def _ptrs(ts, dtype=torch.float64, per=1):
    """Host array of device pointers; per = 3 pads each case's list to 3."""
    vals = []
    for t in ts:
        if per == 1:
            vals.append(_ptr(t, dtype).value)
        else:
            for a in range(per):
                vals.append(_ptr(t[a], dtype).value if a < len(t) and t[a] is not None else None)
    return (ctypes.c_void_p * len(vals))(*vals)


class Batch:
    """Contexts whose solves run as one launch per kernel over all cases."""

    def __init__(self, contexts: Sequence[Context], device="cuda", stream: Optional[torch.cuda.Stream] = None):
        lib = load()
        self.lib = lib
        self.contexts = list(contexts)
        n = len(self.contexts)
        opts = self.contexts[0].opts
        nbytes = lib.ebit_batch_workspace_bytes(n, ctypes.byref(opts))
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        aligned = (self.workspace.data_ptr() + 255) // 256 * 256
        hs = (ctypes.c_void_p * n)(*[c.h.value for c in self.contexts])
        h = ctypes.c_void_p()
        st = lib.ebit_batch_create(ctypes.byref(h), n, hs, ctypes.c_void_p(aligned), ctypes.c_size_t(nbytes),
                                   ctypes.c_void_p(self.stream.cuda_stream))
        if st != OK:
            raise EbitError(st, "ebit_batch_create")
        self.h = h
        self.n = n

    def close(self):
        if getattr(self, "h", None):
            self.lib.ebit_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, where):
        if st != OK:
            raise EbitError(st, where, self.lib.ebit_batch_last_error(self.h).decode())

    def _stats(self):
        return (Stats * self.n)()

    def build_coeffs(self, markers, vcols, ccols, dts):
        self._check(self.lib.ebit_batch_build_coeffs(self.h, _ptrs(markers, per=3), _ptrs(vcols, torch.uint8),
                                                     _ptrs(ccols, torch.uint8), (ctypes.c_double * self.n)(*dts)),
                    "ebit_batch_build_coeffs")

    def heat_solve(self, T_star, T, use_guess=False, check=True):
        s = self._stats()
        st = self.lib.ebit_batch_heat_solve(self.h, _ptrs(T_star), _ptrs(T), int(use_guess), s)
        if check:
            self._check(st, "ebit_batch_heat_solve")
        return [x.as_dict() for x in s]

    def mass_flux(self, T, mdot, stats=True):
        """Per-case mdot; with stats=False the call does not wait for the
        device and returns None."""
        s = self._stats() if stats else None
        self._check(self.lib.ebit_batch_mass_flux(self.h, _ptrs(T), _ptrs(mdot), s), "ebit_batch_mass_flux")
        return [x.as_dict() for x in s] if stats else None

    def autotune(self, b_heat=None, b_press=None, x=None):
        """Batch counterpart of Context.autotune (per-case lists)."""
        o = Opts()
        ms = ctypes.c_double()
        ref = b_heat if b_heat is not None else b_press
        if x is None:
            x = [torch.empty_like(t) for t in ref]
        self._check(self.lib.ebit_batch_autotune(self.h, _ptrs(b_heat) if b_heat is not None else None,
                                                 _ptrs(b_press) if b_press is not None else None, _ptrs(x),
                                                 ctypes.byref(o), ctypes.byref(ms)), "ebit_batch_autotune")
        return {k: getattr(o, k) for k, _ in Opts._fields_}, ms.value

    def autotune_cached(self, path, b_heat=None, b_press=None, x=None):
        """Batch counterpart of Context.autotune_cached."""
        o = Opts()
        ms = ctypes.c_double()
        hit = ctypes.c_int()
        ref = b_heat if b_heat is not None else b_press
        if x is None:
            x = [torch.empty_like(t) for t in ref]
        self._check(self.lib.ebit_batch_autotune_cached(self.h, str(path).encode(),
                                                        _ptrs(b_heat) if b_heat is not None else None,
                                                        _ptrs(b_press) if b_press is not None else None, _ptrs(x),
                                                        ctypes.byref(o), ctypes.byref(ms), ctypes.byref(hit)),
                    "ebit_batch_autotune_cached")
        return {k: getattr(o, k) for k, _ in Opts._fields_}, ms.value, bool(hit.value)

    def project(self, u_l, u_v, mdot, p, use_guess=False, check=True):
        s = self._stats()
        st = self.lib.ebit_batch_project(self.h, _ptrs(u_l, per=3), _ptrs(u_v, per=3), _ptrs(mdot), _ptrs(p),
                                         int(use_guess), s)
        if check:
            self._check(st, "ebit_batch_project")
        return [x.as_dict() for x in s]


# ---------------------------------------------------------------------------
# marshalling of a seeded synthetic case (ebit_inputs.Case) onto the device
# ---------------------------------------------------------------------------
class DeviceCase:
    """Device copies of one case's inputs (plain tensor copies, no arithmetic)."""

    def __init__(self, case, device="cuda"):
        t = lambda a, dt=torch.float64: torch.as_tensor(a, dtype=dt).contiguous().to(device)
        self.case = case
        self.markers = [t(m) for m in case.markers]
        self.vcol = t(case.vcol, torch.uint8)
        self.ccol = t(case.ccol, torch.uint8)
        self.T0 = t(case.T0)
        self.u_l = [t(u) for u in case.u_l]
        self.u_v = [t(u) for u in case.u_v]
        self.grid = make_grid(case.dim, case.n, case.h, case.T_bc, case.p_bc)
        self.props = make_props(case.props)


def context_for(case, opts=None, device="cuda"):
    dc = DeviceCase(case, device)
    ctx = Context(dc.grid, dc.props, opts, device)
    return ctx, dc
