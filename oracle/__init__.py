"""FP64 CPU oracle for list-mode multi-energy-window OSEM SPECT (arXiv 2305.17111).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no code
with the GPU library: the model arithmetic lives in ``lmmew_oracle.c`` (plain C,
double precision) and this module only marshals numpy arrays into it, plus the
exact-model event sampler, whose probabilities come from the C code and whose
random draws come from numpy's PCG64.

Every function in the C file cites the passage of the paper it follows.  The
system parameters arrive as any object with the attributes of ``or_sys`` (see
``SysParams`` below); the oracle does not import the input generators.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lmmew_oracle.c")
_SRC3 = os.path.join(_HERE, "lmmew_oracle3.c")
_LIB = os.path.join(_HERE, "liblmmew_oracle.so")
_lib = None

MAXL = 8
MAXW = 8


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (OpenMP, -O2, strict IEEE: no -ffast-math)."""
    stale = (not os.path.exists(_LIB) or
             os.path.getmtime(_LIB) < max(os.path.getmtime(f) for f in (_SRC, _SRC3)))
    if force or stale:
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
               "-o", tmp, _SRC, _SRC3, "-lm"]
        subprocess.run(cmd, check=True, cwd=_HERE)
        os.replace(tmp, _LIB)
    return _LIB


class _Sys(C.Structure):
    _fields_ = [
        ("n", C.c_int), ("pix", C.c_double), ("ns", C.c_int),
        ("nb", C.c_int), ("na", C.c_int),
        ("fwhm0", C.c_double), ("fwhm_slope", C.c_double), ("dtheta", C.c_double),
        ("nw", C.c_int), ("E", C.c_double * MAXL), ("alpha", C.c_double * MAXL),
        ("nwin", C.c_int), ("wlo", C.c_double * MAXW), ("whi", C.c_double * MAXW),
        ("eres_frac", C.c_double), ("eres_ref", C.c_double),
        ("mu_ref", C.c_double), ("mu_pow", C.c_double),
        ("T", C.c_double), ("me", C.c_double),
    ]


class _Geom(C.Structure):
    _fields_ = [
        ("S", _Sys), ("R", C.c_double), ("hs", C.c_double), ("db", C.c_double),
        ("Q", C.c_int),
        ("mu", C.POINTER(C.c_double)), ("support", C.POINTER(C.c_uint8)),
        ("nsc", C.c_int),
        ("sx", C.POINTER(C.c_double)), ("sy", C.POINTER(C.c_double)),
        ("smu", C.POINTER(C.c_double)),
        ("g_qa", C.POINTER(C.c_double)), ("g_qs", C.POINTER(C.c_double)),
        ("g_sa", C.POINTER(C.c_double)),
        ("Zw", C.c_double * MAXL),
    ]


class _Sys3(C.Structure):
    _fields_ = [("S", _Sys), ("nz", C.c_int), ("nsz", C.c_int), ("nbz", C.c_int),
                ("domega", C.c_double)]


class _Geom3(C.Structure):
    _fields_ = [
        ("S3", _Sys3), ("R", C.c_double), ("Zh", C.c_double), ("hs", C.c_double),
        ("hz", C.c_double), ("db", C.c_double), ("dbz", C.c_double), ("Q", C.c_int),
        ("mu", C.POINTER(C.c_double)), ("support", C.POINTER(C.c_uint8)),
        ("nsc", C.c_int),
        ("sx", C.POINTER(C.c_double)), ("sy", C.POINTER(C.c_double)),
        ("sz", C.POINTER(C.c_double)), ("smu", C.POINTER(C.c_double)),
        ("g_qa", C.POINTER(C.c_double)), ("g_qs", C.POINTER(C.c_double)),
        ("g_sa", C.POINTER(C.c_double)),
        ("Zw", C.c_double * MAXL),
    ]


_D = C.POINTER(C.c_double)
_I = C.POINTER(C.c_int)
_L = C.POINTER(C.c_long)
_G = C.POINTER(_Geom)
_S = C.POINTER(_Sys)
_G3 = C.POINTER(_Geom3)
_S3 = C.POINTER(_Sys3)


def lib():
    global _lib
    if _lib is None:
        build(force=False)            # compiles when missing or older than the sources
        L = C.CDLL(_LIB)
        sig = {
            "or_threads": (C.c_int, []),
            "or_set_threads": (None, [C.c_int]),
            "or_angle_dir": (None, [C.c_int, C.c_int, _D, _D]),
            "or_segment_integral": (C.c_double, [_D, C.c_int, C.c_double, C.c_double,
                                                 C.c_double, C.c_double, C.c_double]),
            "or_Phi_diff": (C.c_double, [C.c_double, C.c_double]),
            "or_kn_K": (C.c_double, [C.c_double, C.c_double, C.c_double]),
            "or_kn_Z": (C.c_double, [C.c_double, C.c_double]),
            "or_sigmaE": (C.c_double, [_S, C.c_double]),
            "or_gauss": (C.c_double, [C.c_double, C.c_double, C.c_double]),
            "or_acc": (C.c_double, [_S, C.c_double]),
            "or_mu_scale": (C.c_double, [_S, C.c_double]),
            "or_psf_sigma": (C.c_double, [_S, C.c_double]),
            "or_psf_bin": (C.c_double, [_G, C.c_int, C.c_double, C.c_double, C.c_int]),
            "or_psf_total": (C.c_double, [_G, C.c_double, C.c_double, C.c_int]),
            "or_psf_density": (C.c_double, [_G, C.c_double, C.c_double, C.c_double, C.c_int]),
            "or_geom_build": (C.c_int, [_G, _S, _D, C.POINTER(C.c_uint8)]),
            "or_geom_free": (None, [_G]),
            "or_Pp": (C.c_double, [_G, C.c_int, C.c_int, C.c_int]),
            "or_Ps": (C.c_double, [_G, C.c_int, C.c_int, C.c_int, C.c_int, _D]),
            "or_event_row": (None, [_G, C.c_int, C.c_int, C.c_double, _D]),
            "or_event_row_scatter": (None, [_G, C.c_int, C.c_int, C.c_double, _D]),
            "or_event_row_pos": (None, [_G, C.c_double, C.c_int, C.c_double, _D]),
            "or_sens_qa": (C.c_double, [_G, C.c_int, C.c_int]),
            "or_sensitivity": (None, [_G, C.c_int, _D]),
            "or_sensitivity_subset": (None, [_G, C.c_int, C.c_int, _D]),
            "or_sample_masses": (C.c_long, [_G, _D, _D]),
            "or_check_events": (C.c_int, [_G, C.c_long, _I, _D, _I, _D]),
            "or_forward": (None, [_G, C.c_long, _I, _D, _I, _D, _D, _D]),
            "or_backproject": (None, [_G, C.c_long, _I, _D, _I, _D, _D, _D]),
            "or_osem": (C.c_int, [_G, C.c_long, _I, _D, _I, _D, C.c_int, C.c_int, _D, _D,
                                  _D, _D, _L]),
            "or3_segment_integral": (C.c_double, [_D, C.c_int, C.c_int, C.c_double]
                                     + [C.c_double] * 6),
            "or3_kn_Z": (C.c_double, [C.c_double, C.c_double]),
            "or3_geom_build": (C.c_int, [_G3, _S3, _D, C.POINTER(C.c_uint8)]),
            "or3_geom_free": (None, [_G3]),
            "or3_voxel_centre": (None, [_G3, C.c_int, _D, _D, _D]),
            "or3_Pp": (C.c_double, [_G3, C.c_int, C.c_int, C.c_int]),
            "or3_Ps": (C.c_double, [_G3, C.c_int, C.c_int, C.c_int, C.c_int, _D]),
            "or3_psf_bin": (C.c_double, [_G3, C.c_int, C.c_int, C.c_double, C.c_double,
                                         C.c_double, C.c_int]),
            "or3_psf_total": (C.c_double, [_G3, C.c_double, C.c_double, C.c_double, C.c_int]),
            "or3_event_row": (None, [_G3, C.c_int, C.c_int, C.c_int, C.c_double, _D]),
            "or3_event_row_scatter": (None, [_G3, C.c_int, C.c_int, C.c_int, C.c_double, _D]),
            "or3_sens_qa": (C.c_double, [_G3, C.c_int, C.c_int]),
            "or3_sensitivity": (None, [_G3, C.c_int, _D]),
            "or3_check_events": (C.c_int, [_G3, C.c_long, _I, _I, _I, _D]),
            "or3_forward": (None, [_G3, C.c_long, _I, _I, _I, _D, _D, _D]),
            "or3_osem": (C.c_int, [_G3, C.c_long, _I, _I, _I, _D, C.c_int, C.c_int, _D, _D,
                                   _D, _D, _L]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(_D)


def _ip(a):
    return a.ctypes.data_as(_I)


def make_sys(p) -> _Sys:
    """Fill the C parameter block from any object carrying the system attributes
    (n, pix, ns, nb, na, fwhm0, fwhm_slope, dtheta, lines, yields, windows,
    eres_frac, eres_ref, mu_ref, mu_pow, T, me)."""
    s = _Sys()
    s.n, s.pix, s.ns, s.nb, s.na = int(p.n), float(p.pix), int(p.ns), int(p.nb), int(p.na)
    s.fwhm0, s.fwhm_slope, s.dtheta = float(p.fwhm0), float(p.fwhm_slope), float(p.dtheta)
    s.nw = len(p.lines)
    for i, (e, y) in enumerate(zip(p.lines, p.yields)):
        s.E[i], s.alpha[i] = float(e), float(y)
    s.nwin = len(p.windows)
    for i, (lo, hi) in enumerate(p.windows):
        s.wlo[i], s.whi[i] = float(lo), float(hi)
    s.eres_frac, s.eres_ref = float(p.eres_frac), float(p.eres_ref)
    s.mu_ref, s.mu_pow = float(p.mu_ref), float(p.mu_pow)
    s.T, s.me = float(p.T), float(p.me)
    return s


# ---- free functions ------------------------------------------------------

def threads():
    """OpenMP threads the oracle uses."""
    return int(lib().or_threads())


def set_threads(n):
    """Threads the oracle's OpenMP loops use from now on."""
    lib().or_set_threads(int(n))


def angle_dir(a, na):
    c, s = C.c_double(), C.c_double()
    lib().or_angle_dir(int(a), int(na), C.byref(c), C.byref(s))
    return c.value, s.value


def segment_integral(mu, n, pix, x0, y0, x1, y1):
    mu = np.ascontiguousarray(mu, dtype=np.float64).ravel()
    return lib().or_segment_integral(_dp(mu), int(n), float(pix), float(x0), float(y0),
                                     float(x1), float(y1))


def kn_K(cosphi, E, me=510.99895):
    return lib().or_kn_K(float(cosphi), float(E), float(me))


def kn_Z(E, me=510.99895):
    return lib().or_kn_Z(float(E), float(me))


def Phi_diff(zhi, zlo):
    return lib().or_Phi_diff(float(zhi), float(zlo))


class Oracle:
    """The model on one attenuation map: tables, rows, sensitivity, OSEM."""

    def __init__(self, params, mu85, mask=None):
        self.params = params
        self.sys = make_sys(params)
        self.mu85 = np.ascontiguousarray(mu85, dtype=np.float64).ravel()
        n = int(params.n)
        assert self.mu85.size == n * n
        self._g = _Geom()
        m = None
        if mask is not None:
            self._mask = np.ascontiguousarray(mask, dtype=np.uint8).ravel()
            m = self._mask.ctypes.data_as(C.POINTER(C.c_uint8))
        rc = lib().or_geom_build(C.byref(self._g), C.byref(self.sys), _dp(self.mu85), m)
        if rc != 0:
            raise ValueError("invalid geometry (n must be a multiple of ns with an even ratio)")
        self.Q = n * n

    def __del__(self):
        try:
            lib().or_geom_free(C.byref(self._g))
        except Exception:
            pass

    # -- geometry accessors
    @property
    def R(self):
        return self._g.R

    @property
    def hs(self):
        return self._g.hs

    @property
    def nsc(self):
        return self._g.nsc

    @property
    def support(self):
        return np.ctypeslib.as_array(self._g.support, shape=(self.Q,)).astype(bool).copy()

    def scatter_points(self):
        k = self._g.nsc
        if k == 0:
            return np.zeros((0, 2)), np.zeros(0)
        xs = np.ctypeslib.as_array(self._g.sx, shape=(k,)).copy()
        ys = np.ctypeslib.as_array(self._g.sy, shape=(k,)).copy()
        mu = np.ctypeslib.as_array(self._g.smu, shape=(k,)).copy()
        return np.stack([xs, ys], 1), mu

    def tables(self):
        na, Q, k = int(self.params.na), self.Q, max(self._g.nsc, 1)
        g_qa = np.ctypeslib.as_array(self._g.g_qa, shape=(na * Q,)).reshape(na, Q).copy()
        g_qs = np.ctypeslib.as_array(self._g.g_qs, shape=(Q * k,)).reshape(Q, k).copy()
        g_sa = np.ctypeslib.as_array(self._g.g_sa, shape=(na * k,)).reshape(na, k).copy()
        return g_qa, g_qs[:, : self._g.nsc], g_sa[:, : self._g.nsc]

    def pixel_centre(self, q):
        n, pix = int(self.params.n), float(self.params.pix)
        return ((q % n) + 0.5) * pix - self.R, ((q // n) + 0.5) * pix - self.R

    # -- model pieces
    def Pp(self, q, a, w):
        return lib().or_Pp(C.byref(self._g), int(q), int(a), int(w))

    def Ps(self, q, si, a, w):
        ep = C.c_double()
        v = lib().or_Ps(C.byref(self._g), int(q), int(si), int(a), int(w), C.byref(ep))
        return v, ep.value

    def psf_bin(self, b, x, y, a):
        return lib().or_psf_bin(C.byref(self._g), int(b), float(x), float(y), int(a))

    def psf_total(self, x, y, a):
        return lib().or_psf_total(C.byref(self._g), float(x), float(y), int(a))

    def psf_density(self, u, x, y, a):
        return lib().or_psf_density(C.byref(self._g), float(u), float(x), float(y), int(a))

    def acc(self, E):
        return lib().or_acc(C.byref(self.sys), float(E))

    def sigmaE(self, E):
        return lib().or_sigmaE(C.byref(self.sys), float(E))

    def mu_scale(self, E):
        return lib().or_mu_scale(C.byref(self.sys), float(E))

    def psf_sigma(self, depth):
        return lib().or_psf_sigma(C.byref(self.sys), float(depth))

    def row(self, b, a, E):
        out = np.zeros(self.Q)
        lib().or_event_row(C.byref(self._g), int(b), int(a), float(E), _dp(out))
        return out

    def row_pos(self, u, a, E):
        """Row of an event recorded at continuous lateral position u (mm)."""
        out = np.zeros(self.Q)
        lib().or_event_row_pos(C.byref(self._g), float(u), int(a), float(E), _dp(out))
        return out

    def row_scatter(self, b, a, E):
        out = np.zeros(self.Q)
        lib().or_event_row_scatter(C.byref(self._g), int(b), int(a), float(E), _dp(out))
        return out

    def sens_qa(self, q, a):
        return lib().or_sens_qa(C.byref(self._g), int(q), int(a))

    def sensitivity(self, nsub):
        out = np.zeros((int(nsub), self.Q))
        lib().or_sensitivity(C.byref(self._g), int(nsub), _dp(out))
        return out

    def sensitivity_subset(self, nsub, s):
        """Row s of sensitivity(nsub), computed alone."""
        out = np.zeros(self.Q)
        lib().or_sensitivity_subset(C.byref(self._g), int(nsub), int(s), _dp(out))
        return out

    # -- events
    @staticmethod
    def _ev(events):
        """Event arrays for the C calls.  A list carries either "bin" (detector
        bins) or "position" (continuous lateral position, mm); one that has
        both is taken as binned."""
        a = np.ascontiguousarray(events["angle"], dtype=np.int32)
        e = np.ascontiguousarray(events["energy"], dtype=np.float64)
        if "bin" in events:
            b = np.ascontiguousarray(events["bin"], dtype=np.int32)
            return b, None, a, e
        u = np.ascontiguousarray(events["position"], dtype=np.float64)
        return None, u, a, e

    @staticmethod
    def _bu(b, u):
        return (_ip(b) if b is not None else None), (_dp(u) if u is not None else None)

    def check_events(self, events):
        b, u, a, e = self._ev(events)
        return lib().or_check_events(C.byref(self._g), a.size, *self._bu(b, u), _ip(a), _dp(e))

    def forward(self, events, lam):
        b, u, a, e = self._ev(events)
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        p = np.zeros(a.size)
        lib().or_forward(C.byref(self._g), a.size, *self._bu(b, u), _ip(a), _dp(e), _dp(lam),
                         _dp(p))
        return p

    def backproject(self, events, wj):
        b, u, a, e = self._ev(events)
        wj = np.ascontiguousarray(wj, dtype=np.float64)
        out = np.zeros(self.Q)
        lib().or_backproject(C.byref(self._g), a.size, *self._bu(b, u), _ip(a), _dp(e), _dp(wj),
                             _dp(out))
        return out

    def osem(self, events, nsub, niter, lam0, sens=None):
        """Returns (final image, history [niter*nsub, Q], ll [niter*nsub], skipped)."""
        b, u, a, e = self._ev(events)
        if sens is None:
            sens = self.sensitivity(nsub)
        sens = np.ascontiguousarray(sens, dtype=np.float64)
        lam = np.array(lam0, dtype=np.float64).copy()
        K = int(nsub) * int(niter)
        hist = np.zeros((K, self.Q))
        ll = np.zeros(K)
        sk = np.zeros(K, dtype=np.int64)
        lib().or_osem(C.byref(self._g), a.size, *self._bu(b, u), _ip(a), _dp(e), int(nsub),
                      int(niter),
                      _dp(sens), _dp(lam), _dp(hist), _dp(ll),
                      sk.ctypes.data_as(_L))
        return lam, hist, ll, sk

    # -- exact-model sampler
    def sample_masses(self, lam):
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        Qm = int(self.support.sum())
        size = Qm * int(self.params.na) * len(self.params.lines) * (1 + self.nsc)
        m = np.zeros(size)
        lib().or_sample_masses(C.byref(self._g), _dp(lam), _dp(m))
        return m

    def sample_events(self, lam, n_events, seed, poisson=False):
        """Events drawn from the normalised model density on the acceptance region.

        Draws (pixel, angle, line, component) from the categorical whose masses
        are lambda_q x path sensitivity x detector probability x window
        acceptance; then the lateral position from the depth-dependent Gaussian
        truncated to the detector, and the energy from the resolution Gaussian
        at the true energy truncated to the windows.  With ``poisson`` the
        count is Poisson with mean ``n_events``.  The result holds both the
        bin and the continuous lateral position ("position", mm) of every
        event; a list handed to the other calls with "bin" removed is taken
        as continuous."""
        p = self.params
        rng = np.random.Generator(np.random.PCG64(seed))
        m = self.sample_masses(lam)
        tot = m.sum()
        J = int(rng.poisson(n_events)) if poisson else int(n_events)
        cdf = np.cumsum(m)
        cdf /= cdf[-1]
        picks = np.searchsorted(cdf, rng.random(J), side="right")
        picks = np.minimum(picks, m.size - 1)
        na, nw, nc = int(p.na), len(p.lines), 1 + self.nsc
        comp = picks % nc
        w = (picks // nc) % nw
        a = (picks // (nc * nw)) % na
        qi = picks // (nc * nw * na)
        qs = np.flatnonzero(self.support)
        q = qs[qi]
        sxy, _ = self.scatter_points()
        bins = np.zeros(J, dtype=np.int32)
        pos = np.zeros(J)
        energies = np.zeros(J)
        db = 2 * self.R / int(p.nb)
        for j in range(J):
            if comp[j] == 0:
                x, y = self.pixel_centre(q[j])
                Et = float(p.lines[w[j]])
            else:
                si = int(comp[j] - 1)
                x, y = sxy[si]
                _, Et = self.Ps(q[j], si, a[j], w[j])
            c, s = angle_dir(a[j], na)
            u0 = -x * s + y * c
            depth = self.R - (x * c + y * s)
            sig = self.psf_sigma(depth)
            while True:
                u = rng.normal(u0, sig)
                if -self.R <= u < self.R:
                    break
            pos[j] = u
            bins[j] = min(int(np.floor((u + self.R) / db)), int(p.nb) - 1)
            se = self.sigmaE(Et)
            while True:
                e = rng.normal(Et, se)
                if any(lo <= e <= hi for lo, hi in p.windows):
                    break
            energies[j] = e
        return {"bin": bins, "position": pos, "angle": a.astype(np.int32), "energy": energies,
                "pixel": q, "line": w, "component": comp, "total_mass": tot}


def segment_integral3(mu, n, nz, pix, x0, y0, z0, x1, y1, z1):
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    return lib().or3_segment_integral(_dp(mu), int(n), int(nz), float(pix), float(x0),
                                      float(y0), float(z0), float(x1), float(y1), float(z1))


def kn_Z3(E, me=510.99895):
    return lib().or3_kn_Z(float(E), float(me))


class Oracle3:
    """The 3-D single-scatter model on one voxelised attenuation map (nz
    slices of n x n; flat index (iz*n + iy)*n + ix): tables, rows,
    sensitivity, OSEM.  Events carry "bin", "bin_z", "angle", "energy"."""

    def __init__(self, params, mu85, mask=None):
        self.params = params
        s3 = _Sys3()
        s3.S = make_sys(params)
        s3.nz, s3.nsz, s3.nbz = int(params.nz), int(params.nsz), int(params.nbz)
        s3.domega = float(params.domega)
        self.sys = s3
        n, nz = int(params.n), int(params.nz)
        self.mu85 = np.ascontiguousarray(mu85, dtype=np.float64).ravel()
        assert self.mu85.size == n * n * nz
        self._g = _Geom3()
        m = None
        if mask is not None:
            self._mask = np.ascontiguousarray(mask, dtype=np.uint8).ravel()
            m = self._mask.ctypes.data_as(C.POINTER(C.c_uint8))
        rc = lib().or3_geom_build(C.byref(self._g), C.byref(self.sys), _dp(self.mu85), m)
        if rc != 0:
            raise ValueError("invalid geometry (n/ns and nz/nsz must be even integers)")
        self.Q = n * n * nz

    def __del__(self):
        try:
            lib().or3_geom_free(C.byref(self._g))
        except Exception:
            pass

    @property
    def R(self):
        return self._g.R

    @property
    def Zh(self):
        return self._g.Zh

    @property
    def nsc(self):
        return self._g.nsc

    @property
    def support(self):
        return np.ctypeslib.as_array(self._g.support, shape=(self.Q,)).astype(bool).copy()

    def scatter_points(self):
        k = self._g.nsc
        if k == 0:
            return np.zeros((0, 3)), np.zeros(0)
        xyz = [np.ctypeslib.as_array(getattr(self._g, f), shape=(k,)).copy()
               for f in ("sx", "sy", "sz")]
        mu = np.ctypeslib.as_array(self._g.smu, shape=(k,)).copy()
        return np.stack(xyz, 1), mu

    def voxel_centre(self, q):
        x, y, z = C.c_double(), C.c_double(), C.c_double()
        lib().or3_voxel_centre(C.byref(self._g), int(q), C.byref(x), C.byref(y), C.byref(z))
        return x.value, y.value, z.value

    def Pp(self, q, a, w):
        return lib().or3_Pp(C.byref(self._g), int(q), int(a), int(w))

    def Ps(self, q, si, a, w):
        ep = C.c_double()
        v = lib().or3_Ps(C.byref(self._g), int(q), int(si), int(a), int(w), C.byref(ep))
        return v, ep.value

    def psf_bin(self, b, bz, x, y, z, a):
        return lib().or3_psf_bin(C.byref(self._g), int(b), int(bz), float(x), float(y),
                                 float(z), int(a))

    def psf_total(self, x, y, z, a):
        return lib().or3_psf_total(C.byref(self._g), float(x), float(y), float(z), int(a))

    def row(self, b, bz, a, E):
        out = np.zeros(self.Q)
        lib().or3_event_row(C.byref(self._g), int(b), int(bz), int(a), float(E), _dp(out))
        return out

    def row_scatter(self, b, bz, a, E):
        out = np.zeros(self.Q)
        lib().or3_event_row_scatter(C.byref(self._g), int(b), int(bz), int(a), float(E),
                                    _dp(out))
        return out

    def sens_qa(self, q, a):
        return lib().or3_sens_qa(C.byref(self._g), int(q), int(a))

    def sensitivity(self, nsub):
        out = np.zeros((int(nsub), self.Q))
        lib().or3_sensitivity(C.byref(self._g), int(nsub), _dp(out))
        return out

    @staticmethod
    def _ev(events):
        b = np.ascontiguousarray(events["bin"], dtype=np.int32)
        bz = np.ascontiguousarray(events["bin_z"], dtype=np.int32)
        a = np.ascontiguousarray(events["angle"], dtype=np.int32)
        e = np.ascontiguousarray(events["energy"], dtype=np.float64)
        return b, bz, a, e

    def check_events(self, events):
        b, bz, a, e = self._ev(events)
        return lib().or3_check_events(C.byref(self._g), a.size, _ip(b), _ip(bz), _ip(a), _dp(e))

    def forward(self, events, lam):
        b, bz, a, e = self._ev(events)
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        p = np.zeros(a.size)
        lib().or3_forward(C.byref(self._g), a.size, _ip(b), _ip(bz), _ip(a), _dp(e),
                          _dp(lam), _dp(p))
        return p

    def osem(self, events, nsub, niter, lam0, sens=None):
        """Returns (final image, history [niter*nsub, Q], ll [niter*nsub], skipped)."""
        b, bz, a, e = self._ev(events)
        if sens is None:
            sens = self.sensitivity(nsub)
        sens = np.ascontiguousarray(sens, dtype=np.float64)
        lam = np.array(lam0, dtype=np.float64).copy()
        K = int(nsub) * int(niter)
        hist = np.zeros((K, self.Q))
        ll = np.zeros(K)
        sk = np.zeros(K, dtype=np.int64)
        lib().or3_osem(C.byref(self._g), a.size, _ip(b), _ip(bz), _ip(a), _dp(e), int(nsub),
                       int(niter), _dp(sens), _dp(lam), _dp(hist), _dp(ll),
                       sk.ctypes.data_as(_L))
        return lam, hist, ll, sk
