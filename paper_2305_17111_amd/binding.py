"""ctypes binding of liblmmew.so: argument marshalling only.

Every entry point of ``include/lmmew.h`` is exposed under the same name through
``Context`` and ``Plan``.  Device arrays are torch tensors on the current HIP
device; work goes to torch's current stream.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "liblmmew.so")

MAX_LINES = 8
MAX_WIN = 8


class LmmewError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"lmmew status {status}: {msg}")
        self.status = status


class _System(C.Structure):
    _fields_ = [
        ("n", C.c_int32), ("ns", C.c_int32), ("n_bins", C.c_int32), ("n_angles", C.c_int32),
        ("n_lines", C.c_int32), ("n_windows", C.c_int32),
        ("pixel_mm", C.c_double), ("psf_fwhm0_mm", C.c_double), ("psf_fwhm_slope", C.c_double),
        ("coll_dtheta", C.c_double),
        ("line_keV", C.c_double * MAX_LINES), ("line_yield", C.c_double * MAX_LINES),
        ("win_lo_keV", C.c_double * MAX_WIN), ("win_hi_keV", C.c_double * MAX_WIN),
        ("eres_frac", C.c_double), ("eres_ref_keV", C.c_double),
        ("mu_ref_keV", C.c_double), ("mu_power", C.c_double),
        ("T", C.c_double), ("electron_keV", C.c_double),
        ("nz", C.c_int32), ("ns_z", C.c_int32), ("n_bins_z", C.c_int32),
        ("coll_solid_angle", C.c_double),
    ]


class _Events(C.Structure):
    _fields_ = [("n", C.c_int64), ("bin", C.c_void_p), ("angle", C.c_void_p),
                ("energy_keV", C.c_void_p), ("position_mm", C.c_void_p),
                ("bin_z", C.c_void_p)]


class _Stats(C.Structure):
    _fields_ = [("skipped_total", C.c_int64), ("skipped", C.POINTER(C.c_int64)),
                ("subset_loglik", C.POINTER(C.c_double))]


_lib = None


def library_path():
    return _LIBPATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIBPATH):
        raise ImportError(f"{_LIBPATH} is missing: build it with __graft_entry__.build() "
                          "(there is no CPU fallback)")
    L = C.CDLL(_LIBPATH)
    vp, i32, i64 = C.c_void_p, C.c_int, C.c_int64
    sig = {
        "lmmew_status_string": (C.c_char_p, [i32]),
        "lmmew_last_error": (C.c_char_p, [vp]),
        "lmmew_create": (i32, [C.POINTER(_System), vp, vp, vp, C.POINTER(vp)]),
        "lmmew_destroy": (i32, [vp]),
        "lmmew_sensitivity": (i32, [vp, i32, vp, vp]),
        "lmmew_forward": (i32, [vp, C.POINTER(_Events), vp, vp, vp]),
        "lmmew_backproject": (i32, [vp, C.POINTER(_Events), vp, vp, vp]),
        "lmmew_plan_create": (i32, [vp, C.POINTER(_Events), vp, i32, i32, vp, C.POINTER(vp)]),
        "lmmew_plan_destroy": (i32, [vp]),
        "lmmew_osem_iter": (i32, [vp, vp, i32, vp, vp, C.POINTER(_Stats), vp]),
        "lmmew_osem_subiter": (i32, [vp, vp, i32, vp, vp, C.POINTER(_Stats), vp]),
        "lmmew_plan_set_event_tile": (i32, [vp, vp, i32, vp]),
        "lmmew_osem_graph": (i32, [vp, vp, i32, vp, vp, vp]),
        "lmmew_autotune": (i32, [vp, vp, i32, vp, C.POINTER(C.c_int)]),
        "lmmew_plan_get_event_tile": (i32, [vp]),
        "lmmew_plan_terms": (i32, [vp, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
        "lmmew_plan_profile": (i32, [vp, vp, i32]),
        "lmmew_rows": (i32, [vp, C.POINTER(_Events), i32, vp, vp]),
        "lmmew_mlp_create": (i32, [vp, C.c_uint64, C.POINTER(vp)]),
        "lmmew_mlp_destroy": (i32, [vp]),
        "lmmew_mlp_get_params": (i32, [vp, vp, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
        "lmmew_mlp_set_params": (i32, [vp, vp, C.c_double, C.c_double]),
        "lmmew_mlp_set_grid": (i32, [vp, i32]),
        "lmmew_set_scatter_pixel_grid": (i32, [vp, i32, vp]),
        "lmmew_scatter_pixel_grid_nodes": (i32, [vp]),
        "lmmew_mlp_grid_nodes": (i32, [vp]),
        "lmmew_mlp_forward": (i32, [vp, vp, vp, i64, vp, vp]),
        "lmmew_mlp_grad": (i32, [vp, vp, vp, vp, i64, vp, C.POINTER(C.c_double), vp]),
        "lmmew_mlp_train": (i32, [vp, vp, vp, vp, i64, i32, i32, C.c_double, C.c_uint64,
                                  C.POINTER(C.c_double), vp]),
        "lmmew_scatter_labels": (i32, [vp, i64, C.c_uint64, vp, vp, vp]),
        "lmmew_mlp_fit": (i32, [vp, vp, i64, i32, i32, C.c_double, C.c_double, C.c_uint64,
                                C.POINTER(C.c_double), vp]),
        "lmmew_mlp_fit_labels": (i32, [vp, vp, vp, vp, i64, i32, i32, C.c_double, C.c_double,
                                       C.c_uint64, C.POINTER(C.c_double), vp]),
        "lmmew_set_scatter_model": (i32, [vp, vp]),
        "lmmew_plan_create_maps": (i32, [vp, vp, vp, i32, i32, vp, vp]),
        "lmmew_plan_profile_read_kernels": (i32, [vp, vp, C.POINTER(C.c_double),
                                                  C.POINTER(C.c_int64)]),
        "lmmew_support_size": (i64, [vp]),
        "lmmew_roi_uptake": (i32, [vp, vp, i32, vp, i32, vp, vp]),
        "lmmew_roi_uptake_noalloc": (i32, [vp, vp, i32, vp, i32, vp, vp]),
        "lmmew_plan_cache_rows": (i32, [vp, vp, i32, vp]),
        "lmmew_path_table": (i32, [vp, i32, vp]),
        "lmmew_path_table_bytes": (i64, [vp]),
        "lmmew_roi_metrics": (i32, [vp, vp, i32, i32, i32, vp, vp, vp]),
        "lmmew_plan_profile_read": (i32, [vp, vp, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
        "lmmew_line_mask": (i32, [C.POINTER(_System), C.c_float]),
        "lmmew_calibrate": (i32, [i32, vp, C.POINTER(C.c_double)]),
        "lmmew_plan_rows": (i32, [vp, vp, i32, vp, i64, vp, vp]),
        "lmmew_psf_table": (i32, [vp, i32, vp]),
        "lmmew_set_scatter_scale": (i32, [vp, C.c_double]),
        "lmmew_set_scatter_scale_windows": (i32, [vp, vp, i32]),
        "lmmew_scatter_scale_fit_windows": (i32, [vp, vp, C.POINTER(_Events), vp, i32, vp]),
        "lmmew_scatter_scale_fit": (i32, [vp, vp, C.POINTER(_Events), C.POINTER(C.c_double), vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def system_from_params(p) -> _System:
    """Fill lmmew_system from any object with the system attributes (n, pix, ns, nb,
    na, fwhm0, fwhm_slope, dtheta, lines, yields, windows, eres_frac, eres_ref,
    mu_ref, mu_pow, T, me; for the 3-D model also nz, nsz, nbz, domega)."""
    s = _System()
    s.n, s.ns, s.n_bins, s.n_angles = int(p.n), int(p.ns), int(p.nb), int(p.na)
    s.n_lines, s.n_windows = len(p.lines), len(p.windows)
    s.pixel_mm, s.psf_fwhm0_mm, s.psf_fwhm_slope = float(p.pix), float(p.fwhm0), float(p.fwhm_slope)
    s.coll_dtheta = float(p.dtheta)
    for i, (e, y) in enumerate(zip(p.lines, p.yields)):
        s.line_keV[i], s.line_yield[i] = float(e), float(y)
    for i, (lo, hi) in enumerate(p.windows):
        s.win_lo_keV[i], s.win_hi_keV[i] = float(lo), float(hi)
    s.eres_frac, s.eres_ref_keV = float(p.eres_frac), float(p.eres_ref)
    s.mu_ref_keV, s.mu_power = float(p.mu_ref), float(p.mu_pow)
    s.T, s.electron_keV = float(p.T), float(p.me)
    nz = int(getattr(p, "nz", 0) or 0)
    if nz > 0:
        s.nz, s.ns_z, s.n_bins_z = nz, int(p.nsz), int(p.nbz)
        s.coll_solid_angle = float(p.domega)
    return s


def line_mask(p, energy_keV):
    """lmmew_line_mask: the lines (bit w: line w) whose scattered terms an event
    of this measured energy keeps under system parameters p (host only)."""
    s = system_from_params(p)
    m = _load().lmmew_line_mask(C.byref(s), C.c_float(energy_keV))
    if m < 0:
        raise LmmewError(m, "lmmew_line_mask: invalid arguments")
    return m


def calibrate(kind):
    """lmmew_calibrate: measured rate on the current device of the per-event
    kernel's term chain (kind 0, terms/s), FP32 FMA (1) or exp2 (2), per second."""
    rate = C.c_double(0.0)
    rc = _load().lmmew_calibrate(int(kind), _stream(), C.byref(rate))
    if rc != 0:
        raise LmmewError(rc, _load().lmmew_status_string(rc).decode())
    return rate.value


def roi_metrics(est, truth):
    """lmmew_roi_metrics: est [S, N, K], truth [S, K] -> (enrmse, bias, std), each [K]."""
    import numpy as np

    est = np.ascontiguousarray(est, np.float64)
    truth = np.ascontiguousarray(truth, np.float64)
    S, N, K = est.shape
    if truth.shape != (S, K):
        raise ValueError("truth must be [S, K]")
    out = [np.zeros(K) for _ in range(3)]
    rc = _load().lmmew_roi_metrics(C.c_void_p(est.ctypes.data), C.c_void_p(truth.ctypes.data),
                                   S, N, K, *[C.c_void_p(o.ctypes.data) for o in out])
    if rc != 0:
        raise LmmewError(rc, "lmmew_roi_metrics: invalid arguments")
    return tuple(out)


def plan_maps(contexts, ev, n_subsets, case_offsets):
    """A plan whose case c uses contexts[c]'s attenuation map
    (lmmew_plan_create_maps); it belongs to contexts[0]."""
    return Plan(contexts[0], ev, n_subsets, case_offsets, maps=contexts)


def events_to_device(ev, device="cuda"):
    """dict(bin, angle, energy) of arrays -> dict of device tensors (int16, int16,
    float32).  A dict without "bin" carries continuous lateral positions in mm
    under "position" (float32 on the device) instead."""
    out = {
        "angle": torch.as_tensor(ev["angle"]).to(device=device, dtype=torch.int16).contiguous(),
        "energy": torch.as_tensor(ev["energy"]).to(device=device, dtype=torch.float32).contiguous(),
    }
    if "bin" in ev:
        out["bin"] = torch.as_tensor(ev["bin"]).to(device=device, dtype=torch.int16).contiguous()
    else:
        out["position"] = torch.as_tensor(ev["position"]).to(device=device,
                                                             dtype=torch.float32).contiguous()
    if "bin_z" in ev:
        out["bin_z"] = torch.as_tensor(ev["bin_z"]).to(device=device,
                                                       dtype=torch.int16).contiguous()
    return out


def _events(ev):
    a, e = ev["angle"], ev["energy"]
    cont = "bin" not in ev
    x = ev["position"] if cont else ev["bin"]
    for t, dt in ((x, torch.float32 if cont else torch.int16), (a, torch.int16),
                  (e, torch.float32)):
        if t.dtype != dt or not t.is_cuda or not t.is_contiguous():
            raise TypeError("events must be contiguous device tensors (bin int16 or position "
                            "float32, angle int16, energy float32)")
    n = a.numel()
    if x.numel() != n or e.numel() != n:
        raise ValueError("event arrays differ in length")
    bz = None
    if "bin_z" in ev:
        z = ev["bin_z"]
        if z.dtype != torch.int16 or not z.is_cuda or not z.is_contiguous() or z.numel() != n:
            raise TypeError("bin_z must be a contiguous int16 device tensor of the events' length")
        bz = z.data_ptr()
    if cont:
        return _Events(n, None, a.data_ptr(), e.data_ptr(), x.data_ptr(), bz)
    return _Events(n, x.data_ptr(), a.data_ptr(), e.data_ptr(), None, bz)


class Context:
    """lmmew_create / lmmew_destroy and the per-map entry points."""

    def __init__(self, params, mu85, support=None):
        L = _load()
        self.params = params
        self.sys = system_from_params(params)
        self.n = int(params.n)
        self.nz = int(getattr(params, "nz", 0) or 0)
        self.Q = self.n * self.n * max(self.nz, 1)
        self.mu85 = torch.as_tensor(mu85).to("cuda", torch.float32).contiguous().view(-1)
        if self.mu85.numel() != self.Q:
            raise ValueError("mu85 must have n*n (3-D: n*n*nz) entries")
        self.support = None
        if support is not None:
            self.support = torch.as_tensor(support).to("cuda", torch.uint8).contiguous().view(-1)
        h = C.c_void_p()
        rc = L.lmmew_create(C.byref(self.sys), _ptr(self.mu85), _ptr(self.support), _stream(),
                            C.byref(h))
        if rc != 0:
            raise LmmewError(rc, L.lmmew_status_string(rc).decode())
        self._h = h

    def _check(self, rc):
        if rc != 0:
            L = _load()
            raise LmmewError(rc, L.lmmew_last_error(self._h).decode() or
                             L.lmmew_status_string(rc).decode())

    def close(self):
        if getattr(self, "_h", None):
            _load().lmmew_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def lmmew_sensitivity(self, n_subsets, out=None):
        if out is None:
            out = torch.empty((n_subsets, self.Q), device="cuda", dtype=torch.float32)
        self._check(_load().lmmew_sensitivity(self._h, int(n_subsets), _ptr(out), _stream()))
        return out

    def lmmew_forward(self, ev, lam, out=None):
        e = _events(ev)
        lam = lam.contiguous()
        if out is None:
            out = torch.empty(e.n, device="cuda", dtype=torch.float32)
        self._check(_load().lmmew_forward(self._h, C.byref(e), _ptr(lam), _ptr(out), _stream()))
        return out

    def lmmew_backproject(self, ev, w, out=None):
        e = _events(ev)
        w = w.contiguous()
        if out is None:
            out = torch.empty(self.Q, device="cuda", dtype=torch.float32)
        self._check(_load().lmmew_backproject(self._h, C.byref(e), _ptr(w), _ptr(out), _stream()))
        return out

    def lmmew_rows(self, ev, part=0, out=None):
        """Full rows a_jq [n, n*n]; part 0 context model, 1 exact scattered, 2 unscattered,
        3 exact."""
        e = _events(ev)
        if out is None:
            out = torch.empty((e.n, self.Q), device="cuda", dtype=torch.float32)
        self._check(_load().lmmew_rows(self._h, C.byref(e), int(part), _ptr(out), _stream()))
        return out

    def set_scatter_pixel_grid(self, grid):
        """Exact model: scattered part at node pixels every `grid` pixels,
        interpolated to the support (1: every pixel)."""
        self._check(_load().lmmew_set_scatter_pixel_grid(self._h, int(grid), _stream()))

    def scatter_pixel_grid_nodes(self):
        n = _load().lmmew_scatter_pixel_grid_nodes(self._h)
        self._check(min(n, 0))
        return n

    @property
    def support_size(self):
        return int(_load().lmmew_support_size(self._h))

    def lmmew_scatter_labels(self, n_events, seed):
        """(feats [n_events*Qm, 6], raw [n_events*Qm]) from the exact scatter model."""
        Qm = self.support_size
        feats = torch.empty((n_events * Qm, 6), device="cuda", dtype=torch.float32)
        raw = torch.empty(n_events * Qm, device="cuda", dtype=torch.float32)
        self._check(_load().lmmew_scatter_labels(self._h, int(n_events), C.c_uint64(seed),
                                                 _ptr(feats), _ptr(raw), _stream()))
        return feats, raw

    def lmmew_set_scatter_model(self, mlp):
        self._check(_load().lmmew_set_scatter_model(self._h, mlp._h if mlp is not None else None))
        self._scatter_model = mlp

    def lmmew_set_scatter_scale(self, scale):
        self._check(_load().lmmew_set_scatter_scale(self._h, float(scale)))

    def lmmew_scatter_scale_fit(self, mlp, ev):
        """Exact over network once-scattered density summed over the events' rows."""
        e = _events(ev)
        out = C.c_double()
        self._check(_load().lmmew_scatter_scale_fit(self._h, mlp._h, C.byref(e), C.byref(out),
                                                    _stream()))
        return out.value

    def lmmew_set_scatter_scale_windows(self, scales):
        import numpy as np

        v = np.ascontiguousarray(scales, np.float64)
        self._check(_load().lmmew_set_scatter_scale_windows(self._h, C.c_void_p(v.ctypes.data),
                                                            int(v.size)))

    def lmmew_scatter_scale_fit_windows(self, mlp, ev):
        """lmmew_scatter_scale_fit per energy window (numpy array, one per window)."""
        import numpy as np

        e = _events(ev)
        out = np.zeros(len(self.params.windows), np.float64)
        self._check(_load().lmmew_scatter_scale_fit_windows(
            self._h, mlp._h, C.byref(e), C.c_void_p(out.ctypes.data), int(out.size), _stream()))
        return out

    set_scatter_scale = lmmew_set_scatter_scale
    scatter_scale_fit = lmmew_scatter_scale_fit
    set_scatter_scale_windows = lmmew_set_scatter_scale_windows
    scatter_scale_fit_windows = lmmew_scatter_scale_fit_windows

    def lmmew_mlp_create(self, seed=0):
        return Mlp(self, seed)

    def lmmew_roi_uptake(self, lam, masks, noalloc=False):
        """[n_cases, n_rois] FP64 host array of region sums of lam ([n_cases, Q] or [Q])
        over masks ([n_rois, Q], nonzero = inside).  noalloc selects
        lmmew_roi_uptake_noalloc (static device scratch, no allocation)."""
        import numpy as np

        lam = lam.contiguous()
        m = torch.as_tensor(masks).to("cuda", torch.uint8).contiguous()
        nc = 1 if lam.dim() == 1 else lam.shape[0]
        nk = 1 if m.dim() == 1 else m.shape[0]
        out = np.zeros((nc, nk), np.float64)
        fn = _load().lmmew_roi_uptake_noalloc if noalloc else _load().lmmew_roi_uptake
        self._check(fn(self._h, _ptr(lam), nc, _ptr(m), nk, C.c_void_p(out.ctypes.data),
                       _stream()))
        return out

    def lmmew_roi_uptake_noalloc(self, lam, masks):
        return self.lmmew_roi_uptake(lam, masks, noalloc=True)

    def lmmew_path_table(self, enable=True):
        """Builds (or frees) the context's scatter-path parameter table."""
        self._check(_load().lmmew_path_table(self._h, int(bool(enable)), _stream()))

    def lmmew_psf_table(self, enable=True):
        """Builds (or frees, and stops building) the unscattered bin-probability
        table; returns whether it is in use."""
        rc = _load().lmmew_psf_table(self._h, int(bool(enable)), _stream())
        if rc < 0:
            self._check(rc)
        return bool(rc)

    psf_table = lmmew_psf_table

    @property
    def path_table_bytes(self):
        return int(_load().lmmew_path_table_bytes(self._h))

    path_table = lmmew_path_table
    roi_uptake = lmmew_roi_uptake
    rows = lmmew_rows
    scatter_labels = lmmew_scatter_labels
    set_scatter_model = lmmew_set_scatter_model
    mlp = lmmew_mlp_create

    def lmmew_plan_create(self, ev, n_subsets, case_offsets=None):
        return Plan(self, ev, n_subsets, case_offsets)

    # short aliases
    sensitivity = lmmew_sensitivity
    forward = lmmew_forward
    backproject = lmmew_backproject
    plan = lmmew_plan_create


class Plan:
    """lmmew_plan_create / lmmew_osem_iter / lmmew_plan_destroy.

    With ``maps`` (a list of Context, one per case, maps[0] is ctx) the plan
    comes from lmmew_plan_create_maps and sens is [n_cases][n_subsets][n*n]."""

    def __init__(self, ctx: Context, ev, n_subsets, case_offsets=None, maps=None):
        L = _load()
        self.ctx = ctx
        e = _events(ev)
        self.n_subsets = int(n_subsets)
        if case_offsets is None:
            self.n_cases = 1
            offs = None
        else:
            arr = (C.c_int64 * len(case_offsets))(*[int(x) for x in case_offsets])
            self.n_cases = len(case_offsets) - 1
            offs = C.cast(arr, C.c_void_p)
        h = C.c_void_p()
        if maps is None:
            ctx._check(L.lmmew_plan_create(ctx._h, C.byref(e), offs, self.n_cases,
                                           self.n_subsets, _stream(), C.byref(h)))
        else:
            if len(maps) != self.n_cases or maps[0] is not ctx:
                raise ValueError("maps must hold one context per case, maps[0] the plan's")
            self.maps = list(maps)             # kept alive with the plan
            hs = (C.c_void_p * len(maps))(*[m._h.value for m in maps])
            ctx._check(L.lmmew_plan_create_maps(C.cast(hs, C.c_void_p), C.byref(e), offs,
                                                self.n_cases, self.n_subsets, _stream(),
                                                C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _load().lmmew_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def lmmew_osem_iter(self, n_iters, sens, lam, stats=False):
        """Runs n_iters OSEM iterations in place on lam ([n_cases, Q] or [Q]).
        With stats=True returns (skipped per sub-iteration, subset log-likelihoods)."""
        L = _load()
        st = None
        if stats:
            K = int(n_iters) * self.n_subsets
            sk = (C.c_int64 * max(K, 1))()
            ll = (C.c_double * max(K, 1))()
            st = _Stats(0, C.cast(sk, C.POINTER(C.c_int64)), C.cast(ll, C.POINTER(C.c_double)))
        self.ctx._check(L.lmmew_osem_iter(self.ctx._h, self._h, int(n_iters), _ptr(sens), _ptr(lam),
                                          C.byref(st) if st is not None else None, _stream()))
        if stats:
            return list(sk)[:K], list(ll)[:K]
        return None

    def lmmew_osem_subiter(self, subset, sens, lam, stats=False):
        """One sub-iteration for `subset` in place on lam.  With stats=True returns
        (skipped, subset log-likelihood)."""
        L = _load()
        st = None
        if stats:
            sk = (C.c_int64 * 1)()
            ll = (C.c_double * 1)()
            st = _Stats(0, C.cast(sk, C.POINTER(C.c_int64)), C.cast(ll, C.POINTER(C.c_double)))
        self.ctx._check(L.lmmew_osem_subiter(self.ctx._h, self._h, int(subset), _ptr(sens),
                                             _ptr(lam), C.byref(st) if st is not None else None,
                                             _stream()))
        if stats:
            return sk[0], ll[0]
        return None

    def lmmew_osem_graph(self, n_iters, sens, lam):
        """n_iters iterations as one captured hipGraph launch (replayed on later calls
        with the same arguments)."""
        self.ctx._check(_load().lmmew_osem_graph(self.ctx._h, self._h, int(n_iters), _ptr(sens),
                                                 _ptr(lam), _stream()))

    def lmmew_autotune(self, use_cache=True):
        """Times the per-event kernel at event tiles 16/32/64 and keeps the fastest."""
        ch = C.c_int()
        self.ctx._check(_load().lmmew_autotune(self.ctx._h, self._h, int(bool(use_cache)),
                                               _stream(), C.byref(ch)))
        return ch.value

    def lmmew_plan_cache_rows(self, enable=True):
        """Computes every subset's rows once and keeps them (cached-row mode);
        enable=False frees them."""
        self.ctx._check(_load().lmmew_plan_cache_rows(self.ctx._h, self._h, int(bool(enable)),
                                                      _stream()))

    def lmmew_plan_rows(self, subset, events):
        """Rows [len(events), n*n] of the given input events (all of subset `subset`)
        from that sub-iteration's system-model launch."""
        import numpy as np

        idx = np.ascontiguousarray(events, dtype=np.int64)
        rows = torch.empty((idx.size, self.ctx.Q), device="cuda", dtype=torch.float32)
        self.ctx._check(_load().lmmew_plan_rows(self.ctx._h, self._h, int(subset),
                                                C.c_void_p(idx.ctypes.data), int(idx.size),
                                                _ptr(rows), _stream()))
        return rows

    osem_graph = lmmew_osem_graph
    autotune = lmmew_autotune
    cache_rows = lmmew_plan_cache_rows
    rows = lmmew_plan_rows

    def set_event_tile(self, jt):
        self.ctx._check(_load().lmmew_plan_set_event_tile(self.ctx._h, self._h, int(jt), _stream()))

    @property
    def event_tile(self):
        return _load().lmmew_plan_get_event_tile(self._h)

    def lmmew_plan_profile(self, enable=True):
        self.ctx._check(_load().lmmew_plan_profile(self.ctx._h, self._h, int(bool(enable))))

    def lmmew_plan_profile_read(self):
        """(summed duration in ms, number of launches) of the per-event kernel since the
        last read."""
        ms, n = C.c_double(), C.c_int64()
        self.ctx._check(_load().lmmew_plan_profile_read(self.ctx._h, self._h, C.byref(ms),
                                                        C.byref(n)))
        return ms.value, n.value

    def lmmew_plan_profile_read_kernels(self):
        """{kernel: (summed ms, launches)} for the per-event kernel ("k_row") and
        the surrogate ("k_mlp_rows") since the last read."""
        ms = (C.c_double * 2)()
        n = (C.c_int64 * 2)()
        self.ctx._check(_load().lmmew_plan_profile_read_kernels(
            self.ctx._h, self._h, C.cast(ms, C.POINTER(C.c_double)),
            C.cast(n, C.POINTER(C.c_int64))))
        return {"k_row": (ms[0], n[0]), "k_mlp_rows": (ms[1], n[1])}

    profile = lmmew_plan_profile
    profile_read = lmmew_plan_profile_read
    profile_read_kernels = lmmew_plan_profile_read_kernels

    def terms(self):
        t, f = C.c_double(), C.c_double()
        self.ctx._check(_load().lmmew_plan_terms(self._h, C.byref(t), C.byref(f)))
        return t.value, f.value

    osem_iter = lmmew_osem_iter
    osem_subiter = lmmew_osem_subiter


class Mlp:
    """lmmew_mlp_*: the scatter surrogate network of a context."""

    NPARAM = 34049

    def __init__(self, ctx: Context, seed=0):
        self.ctx = ctx
        h = C.c_void_p()
        ctx._check(_load().lmmew_mlp_create(ctx._h, C.c_uint64(seed), C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _load().lmmew_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self):
        import numpy as np

        p = np.zeros(self.NPARAM, np.float32)
        c0, fl = C.c_double(), C.c_double()
        self.ctx._check(_load().lmmew_mlp_get_params(self._h, C.c_void_p(p.ctypes.data),
                                                     C.byref(c0), C.byref(fl)))
        return p, c0.value, fl.value

    def set_params(self, params, c0=0.0, floor=0.0):
        import numpy as np

        p = np.ascontiguousarray(params, np.float32)
        assert p.size == self.NPARAM
        self.ctx._check(_load().lmmew_mlp_set_params(self._h, C.c_void_p(p.ctypes.data),
                                                     float(c0), float(floor)))

    def set_grid(self, grid):
        """Evaluate the network at nodes every `grid` pixels in OSEM and the
        row calls, support pixels interpolated bilinearly (1: every pixel)."""
        self.ctx._check(_load().lmmew_mlp_set_grid(self._h, int(grid)))

    def grid_nodes(self):
        """Positions per event row at which the network is evaluated."""
        n = _load().lmmew_mlp_grid_nodes(self._h)
        self.ctx._check(min(n, 0))
        return n

    def forward(self, feats):
        feats = feats.contiguous()
        y = torch.empty(feats.shape[0], device="cuda", dtype=torch.float32)
        self.ctx._check(_load().lmmew_mlp_forward(self.ctx._h, self._h, _ptr(feats),
                                                  feats.shape[0], _ptr(y), _stream()))
        return y

    def grad(self, feats, target):
        feats, target = feats.contiguous(), target.contiguous()
        g = torch.empty(self.NPARAM, device="cuda", dtype=torch.float32)
        loss = C.c_double()
        self.ctx._check(_load().lmmew_mlp_grad(self.ctx._h, self._h, _ptr(feats), _ptr(target),
                                               feats.shape[0], _ptr(g), C.byref(loss), _stream()))
        return g, loss.value

    def train(self, feats, target, batch=4096, epochs=1, lr=1e-3, seed=0):
        feats, target = feats.contiguous(), target.contiguous()
        losses = (C.c_double * max(epochs, 1))()
        self.ctx._check(_load().lmmew_mlp_train(self.ctx._h, self._h, _ptr(feats), _ptr(target),
                                                feats.shape[0], int(batch), int(epochs), float(lr),
                                                C.c_uint64(seed), losses, _stream()))
        return list(losses)[:epochs]

    def fit(self, n_label_events, epochs=4, batch=4096, lr=1e-3, floor_frac=1e-2, seed=0):
        losses = (C.c_double * max(epochs, 1))()
        self.ctx._check(_load().lmmew_mlp_fit(self.ctx._h, self._h, int(n_label_events),
                                              int(epochs), int(batch), float(lr),
                                              float(floor_frac), C.c_uint64(seed), losses,
                                              _stream()))
        return list(losses)[:epochs]

    def fit_labels(self, feats, raw, epochs=4, batch=4096, lr=1e-3, floor_frac=1e-2, seed=0):
        """lmmew_mlp_fit_labels on device labels (feats [n, 6], raw [n])."""
        feats, raw = feats.contiguous(), raw.contiguous()
        losses = (C.c_double * max(epochs, 1))()
        self.ctx._check(_load().lmmew_mlp_fit_labels(self.ctx._h, self._h, _ptr(feats), _ptr(raw),
                                                     raw.numel(), int(epochs), int(batch),
                                                     float(lr), float(floor_frac),
                                                     C.c_uint64(seed), losses, _stream()))
        return list(losses)[:epochs]

    def fit_maps(self, mu_maps, n_label_events, epochs=4, batch=4096, lr=1e-3, floor_frac=1e-2,
                 seed=0):
        """Trains on labels of several attenuation maps of the same system:
        n_label_events events per map (lmmew_scatter_labels on a context per
        map, seeds seed + k), then lmmew_mlp_fit_labels on all of them."""
        chunks = []
        for k, m in enumerate(mu_maps):
            c = Context(self.ctx.params, torch.as_tensor(m))
            chunks.append(c.scatter_labels(n_label_events, seed + k))
            c.close()
        feats = torch.cat([f for f, _ in chunks])
        raw = torch.cat([r for _, r in chunks])
        del chunks
        return self.fit_labels(feats, raw, epochs, batch, lr, floor_frac, seed)
