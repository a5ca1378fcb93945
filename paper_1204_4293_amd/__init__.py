"""Python binding of the MI355X aperture-mass library (libamap.so).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  Tensors are PyTorch CUDA (ROCm) tensors, contiguous, float32 or
float64; work is enqueued on torch's current stream.  The binding fails with
an exception when the library has not been built or cannot be loaded -- it
has no fallback.

The names mirror the C ABI in include/amap.h.
"""
import ctypes
import os
import re

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB_PATH = os.path.join(HERE, "libamap.so")
HEADER = os.path.join(ROOT, "include", "amap.h")

F32, F64 = 0, 1
FILTER_STARLET, FILTER_S98, FILTER_JBJ04 = 0, 1, 2
BC_PERIODIC, BC_MIRROR, BC_ZERO = 0, 1, 2
_STATUS = {0: "AMAP_OK", 1: "AMAP_E_INVAL", 2: "AMAP_E_NOMEM", 3: "AMAP_E_HIP",
           4: "AMAP_E_UNSUPPORTED", 5: "AMAP_E_BUSY"}
E_NOMEM, E_BUSY = 2, 5

_lib = None


class AmapError(RuntimeError):
    """A non-OK status from the library; ``status`` holds the code."""

    def __init__(self, status, msg):
        super().__init__("%s: %s" % (_STATUS.get(status, status), msg))
        self.status = status


class AmapJob(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("J", ctypes.c_int), ("n_real", ctypes.c_int),
                ("seed", ctypes.c_uint64), ("threshold", ctypes.c_double),
                ("g1", ctypes.c_void_p), ("g2", ctypes.c_void_p),
                ("kappa_e", ctypes.c_void_p), ("planes", ctypes.c_void_p),
                ("sigma", ctypes.c_void_p), ("snr", ctypes.c_void_p),
                ("peaks", ctypes.c_void_p)]


def header_symbols():
    """Names of the functions include/amap.h declares."""
    with open(HEADER) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(amap_[a-z0-9_]+)\s*\(", text)))


def load():
    """Load libamap.so (raises if it is missing: there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libamap.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    P, I, D, U64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_uint64
    sig = {
        "amap_create": (I, [I, ctypes.POINTER(P)]),
        "amap_destroy": (I, [P]),
        "amap_last_error": (ctypes.c_char_p, []),
        "amap_sync": (I, [P, P]),
        "amap_workspace_bytes": (ctypes.c_size_t, [P]),
        "amap_timing_enable": (I, [P, I]),
        "amap_set_autotune": (I, [P, I]),
        "amap_plans_read": (I, [P, ctypes.c_char_p, ctypes.c_size_t]),
        "amap_plans_load": (I, [P, ctypes.c_char_p]),
        "amap_timing_read": (I, [P, ctypes.c_char_p, ctypes.c_size_t, I]),
        "amap_timing_select": (I, [P, ctypes.c_char_p]),
        "amap_ks_invert": (I, [P, I, I, P, P, P, P, P]),
        "amap_ks_invert_noalloc": (I, [P, I, I, P, P, P, P, P]),
        "amap_starlet_forward": (I, [P, I, I, I, P, P, P]),
        "amap_starlet_forward_bc": (I, [P, I, I, I, I, I, P, P, P]),
        "amap_ks_invert_padded": (I, [P, I, I, I, I, P, P, P, P, P]),
        "amap_noise_maps_bc": (I, [P, I, I, I, I, I, I, P, P, I, U64, P, P, P, P]),
        "amap_count_peaks_bc": (I, [P, I, I, I, I, I, P, D, P, P]),
        "amap_count_peaks_masked": (I, [P, I, I, I, I, I, P, P, D, P, P]),
        "amap_mask_shear": (I, [P, I, I, I, P, P, P, P, P, P]),
        "amap_starlet_reconstruct": (I, [P, I, I, I, P, P, P]),
        "amap_map_direct": (I, [P, I, I, P, P, D, I, D, D, P, P]),
        "amap_noise_maps": (I, [P, I, I, I, P, P, I, U64, P, P, P, P]),
        "amap_count_peaks": (I, [P, I, I, I, P, D, P, P]),
        "amap_phase_uniforms": (I, [P, I, U64, U64, P, P]),
        "amap_peak_histogram": (I, [P, I, I, I, P, I, D, D, I, P, P]),
        "amap_plane_moments": (I, [P, I, I, I, P, P, P]),
        "amap_run_path": (I, [P, I, I, I, P, P, I, U64, D, P, P, P, P, P, P, P]),
        "amap_batch_plan": (I, [P, I, ctypes.POINTER(AmapJob), I, ctypes.POINTER(P)]),
        "amap_batch_run": (I, [P, P]),
        "amap_plan_destroy": (I, [P]),
        "amap_job_footprint_bytes": (ctypes.c_size_t, [I, I, I, I]),
        "amap_noise_batch": (I, [I, I]),
        "amap_server_create": (I, [P, I, ctypes.c_size_t, I, I, ctypes.POINTER(P)]),
        "amap_server_submit": (I, [P, ctypes.POINTER(AmapJob), P, ctypes.POINTER(ctypes.c_longlong)]),
        "amap_set_noise_batch": (I, [P, I]),
        "amap_server_poll": (I, [P, ctypes.c_longlong, ctypes.POINTER(I)]),
        "amap_server_wait": (I, [P, ctypes.c_longlong]),
        "amap_server_completed": (I, [P, ctypes.POINTER(ctypes.c_longlong), I, ctypes.POINTER(I)]),
        "amap_server_stats": (I, [P, ctypes.POINTER(I), ctypes.POINTER(I),
                                  ctypes.POINTER(ctypes.c_size_t)]),
        "amap_server_destroy": (I, [P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status):
    if status != 0:
        raise AmapError(status, load().amap_last_error().decode())


def _dt(t):
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.float64:
        return F64
    raise TypeError("tensors must be float32 or float64, got %s" % t.dtype)


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must be on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _side(t):
    n = t.shape[-1]
    if t.shape[-2] != n:
        raise ValueError("maps must be square")
    return n


def job_footprint_bytes(dtype, n, J, n_real):
    return int(load().amap_job_footprint_bytes(dtype, n, J, n_real))


def noise_batch(n, n_real):
    """Realisations per launch sequence of the noise statistics (0: invalid)."""
    return int(load().amap_noise_batch(int(n), int(n_real)))


class Context:
    """A library context on one HIP device (owns twiddles and workspace)."""

    def __init__(self, device=0):
        lib = load()
        h = ctypes.c_void_p()
        _check(lib.amap_create(int(device), ctypes.byref(h)))
        self._h = h
        self.device = torch.device("cuda", device)

    def close(self):
        if self._h:
            load().amap_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sync(self):
        _check(load().amap_sync(self._h, _stream()))

    def plans(self):
        """The context's tuned starlet schedules (list of dicts)."""
        import json
        buf = ctypes.create_string_buffer(1 << 18)
        _check(load().amap_plans_read(self._h, buf, len(buf)))
        return json.loads(buf.value.decode())

    def plans_load(self, plans):
        """Load schedules (a list of dicts as returned by plans(), or its JSON)."""
        import json
        text = plans if isinstance(plans, str) else json.dumps(plans)
        _check(load().amap_plans_load(self._h, text.encode()))

    def set_autotune(self, enable=True):
        """True/1: tuned schedules; False/0: analytic planner; 2: analytic
        planner with sub-grid final noise stages where they apply."""
        mode = int(enable) if not isinstance(enable, bool) else (1 if enable else 0)
        _check(load().amap_set_autotune(self._h, mode))

    def set_noise_batch(self, max_batch=0):
        """Cap the noise realisations per launch sequence (0: the default)."""
        _check(load().amap_set_noise_batch(self._h, int(max_batch)))

    def timing_enable(self, enable=True):
        _check(load().amap_timing_enable(self._h, 1 if enable else 0))

    def timing_select(self, kernel=None):
        """Time only launches named ``kernel`` (None: all)."""
        _check(load().amap_timing_select(self._h, kernel.encode() if kernel else None))

    def timing_read(self, reset=False):
        """{kernel: (launches, total_ms)} of the HIP-event timer."""
        import json
        buf = ctypes.create_string_buffer(1 << 16)
        _check(load().amap_timing_read(self._h, buf, len(buf), 1 if reset else 0))
        return {k: (int(v[0]), float(v[1])) for k, v in json.loads(buf.value.decode()).items()}

    def workspace_bytes(self):
        return int(load().amap_workspace_bytes(self._h))

    def _empty(self, shape, like):
        return torch.empty(shape, dtype=like.dtype, device=like.device)

    def ks_invert(self, g1, g2, kappa_e=None, kappa_b=None, want_b=False):
        n = _side(g1)
        kappa_e = self._empty((n, n), g1) if kappa_e is None else kappa_e
        if kappa_b is None and want_b:
            kappa_b = self._empty((n, n), g1)
        _check(load().amap_ks_invert(self._h, _dt(g1), n, _ptr(g1), _ptr(g2), _ptr(kappa_e),
                                     _ptr(kappa_b), _stream()))
        return kappa_e, kappa_b

    def ks_invert_noalloc(self, g1, g2, kappa_e, kappa_b=None):
        """ks_invert through the entry point that allocates nothing (its
        spectrum in the library's static scratch); outputs must be given."""
        n = _side(g1)
        _check(load().amap_ks_invert_noalloc(self._h, _dt(g1), n, _ptr(g1), _ptr(g2), _ptr(kappa_e),
                                             _ptr(kappa_b), _stream()))
        return kappa_e, kappa_b

    def starlet_forward(self, kappa, J, planes=None):
        n = _side(kappa)
        planes = self._empty((J, n, n), kappa) if planes is None else planes
        _check(load().amap_starlet_forward(self._h, _dt(kappa), n, int(J), _ptr(kappa),
                                           _ptr(planes), _stream()))
        return planes

    def starlet_forward_bc(self, image, J, boundary=BC_MIRROR, planes=None):
        """Starlet planes of an ny x nx field under an edge rule (BC_*)."""
        ny, nx = int(image.shape[-2]), int(image.shape[-1])
        planes = self._empty((J, ny, nx), image) if planes is None else planes
        _check(load().amap_starlet_forward_bc(self._h, _dt(image), ny, nx, int(J), int(boundary),
                                              _ptr(image), _ptr(planes), _stream()))
        return planes

    def ks_invert_padded(self, g1, g2, P, kappa_e=None, kappa_b=None, want_b=False):
        """KS of an ny x nx field zero-extended into a P x P grid."""
        ny, nx = int(g1.shape[-2]), int(g1.shape[-1])
        kappa_e = self._empty((ny, nx), g1) if kappa_e is None else kappa_e
        if kappa_b is None and want_b:
            kappa_b = self._empty((ny, nx), g1)
        _check(load().amap_ks_invert_padded(self._h, _dt(g1), ny, nx, int(P), _ptr(g1), _ptr(g2),
                                            _ptr(kappa_e), _ptr(kappa_b), _stream()))
        return kappa_e, kappa_b

    def noise_maps_bc(self, g1, g2, P, J, boundary, n_real, seed, planes_signal=None,
                      want_snr=True):
        """sigma (and S/N) of an ny x nx field with edges; returns (sigma, snr)."""
        ny, nx = int(g1.shape[-2]), int(g1.shape[-1])
        sigma = self._empty((J - 1, ny, nx), g1)
        snr = self._empty((J - 1, ny, nx), g1) if (want_snr and planes_signal is not None) else None
        _check(load().amap_noise_maps_bc(self._h, _dt(g1), ny, nx, int(P), int(J), int(boundary),
                                         _ptr(g1), _ptr(g2), int(n_real), int(seed),
                                         _ptr(planes_signal), _ptr(sigma), _ptr(snr), _stream()))
        return sigma, snr

    def count_peaks_bc(self, planes, threshold, boundary, counts=None):
        """Peaks above threshold of each ny x nx plane under an edge rule."""
        nplanes, ny, nx = int(planes.shape[0]), int(planes.shape[-2]), int(planes.shape[-1])
        if counts is None:
            counts = torch.empty(nplanes, dtype=torch.int64, device=planes.device)
        _check(load().amap_count_peaks_bc(self._h, _dt(planes), ny, nx, nplanes, int(boundary),
                                          _ptr(planes), float(threshold), _ptr(counts), _stream()))
        return counts

    def count_peaks_masked(self, planes, mask, threshold, boundary, counts=None):
        """Peaks above threshold whose pixel and neighbours are observed
        (mask: uint8 ny x nx, non-zero = observed)."""
        nplanes, ny, nx = int(planes.shape[0]), int(planes.shape[-2]), int(planes.shape[-1])
        if counts is None:
            counts = torch.empty(nplanes, dtype=torch.int64, device=planes.device)
        _check(load().amap_count_peaks_masked(self._h, _dt(planes), ny, nx, nplanes, int(boundary),
                                              _ptr(planes), _ptr(mask), float(threshold), _ptr(counts),
                                              _stream()))
        return counts

    def mask_shear(self, g1, g2, mask, out1=None, out2=None):
        """Shear with missing pixels zeroed; returns (g1_out, g2_out)."""
        ny, nx = int(g1.shape[-2]), int(g1.shape[-1])
        out1 = self._empty((ny, nx), g1) if out1 is None else out1
        out2 = self._empty((ny, nx), g1) if out2 is None else out2
        _check(load().amap_mask_shear(self._h, _dt(g1), ny, nx, _ptr(mask), _ptr(g1), _ptr(g2),
                                      _ptr(out1), _ptr(out2), _stream()))
        return out1, out2

    def starlet_reconstruct(self, planes, out=None):
        J, n = planes.shape[0], _side(planes)
        out = self._empty((n, n), planes) if out is None else out
        _check(load().amap_starlet_reconstruct(self._h, _dt(planes), n, J, _ptr(planes),
                                               _ptr(out), _stream()))
        return out

    def map_direct(self, g1, g2, theta, filter=FILTER_STARLET, fparam=0.0, cut=0.0, out=None):
        n = _side(g1)
        out = self._empty((n, n), g1) if out is None else out
        _check(load().amap_map_direct(self._h, _dt(g1), n, _ptr(g1), _ptr(g2), float(theta),
                                      int(filter), float(fparam), float(cut), _ptr(out), _stream()))
        return out

    def noise_maps(self, g1, g2, J, n_real, seed, planes_signal=None, sigma=None, snr=None,
                   want_snr=True):
        n = _side(g1)
        sigma = self._empty((J - 1, n, n), g1) if sigma is None else sigma
        if snr is None and want_snr and planes_signal is not None:
            snr = self._empty((J - 1, n, n), g1)
        _check(load().amap_noise_maps(self._h, _dt(g1), n, int(J), _ptr(g1), _ptr(g2),
                                      int(n_real), int(seed), _ptr(planes_signal), _ptr(sigma),
                                      _ptr(snr), _stream()))
        return sigma, snr

    def count_peaks(self, snr, threshold, counts=None):
        nplanes, n = snr.shape[0], _side(snr)
        counts = (torch.empty(nplanes, dtype=torch.int64, device=snr.device)
                  if counts is None else counts)
        _check(load().amap_count_peaks(self._h, _dt(snr), n, nplanes, _ptr(snr), float(threshold),
                                       _ptr(counts), _stream()))
        return counts

    def peak_histogram(self, planes, lo, hi, nbins, sign=1, hist=None):
        """Binned peak (sign=+1) or trough (sign=-1) heights per plane."""
        nplanes, n = planes.shape[0], _side(planes)
        hist = (torch.empty((nplanes, nbins), dtype=torch.int64, device=planes.device)
                if hist is None else hist)
        _check(load().amap_peak_histogram(self._h, _dt(planes), n, nplanes, _ptr(planes), int(sign),
                                          float(lo), float(hi), int(nbins), _ptr(hist), _stream()))
        return hist

    def plane_moments(self, planes, out=None):
        """Per plane [mean, m2, m3, m4] (float64, on the device)."""
        nplanes, n = planes.shape[0], _side(planes)
        out = (torch.empty((nplanes, 4), dtype=torch.float64, device=planes.device)
               if out is None else out)
        _check(load().amap_plane_moments(self._h, _dt(planes), n, nplanes, _ptr(planes), _ptr(out),
                                         _stream()))
        return out

    def phase_uniforms(self, n, seed, r, out=None):
        out = torch.empty((n, n), dtype=torch.int32, device=self.device) if out is None else out
        _check(load().amap_phase_uniforms(self._h, int(n), int(seed), int(r), _ptr(out), _stream()))
        return out

    def run_path(self, g1, g2, J, n_real, seed, threshold=3.0, out=None, want_kappa=True):
        """The whole path; returns a dict of output tensors (allocated unless
        given in ``out``)."""
        n = _side(g1)
        o = dict(out or {})
        if want_kappa:
            o.setdefault("kappa_e", self._empty((n, n), g1))
        o.setdefault("planes", self._empty((J, n, n), g1))
        o.setdefault("sigma", self._empty((J - 1, n, n), g1))
        o.setdefault("snr", self._empty((J - 1, n, n), g1))
        o.setdefault("peaks", torch.empty(J - 1, dtype=torch.int64, device=g1.device))
        _check(load().amap_run_path(self._h, _dt(g1), n, int(J), _ptr(g1), _ptr(g2), int(n_real),
                                    int(seed), float(threshold), _ptr(o.get("kappa_e")),
                                    _ptr(o.get("kappa_b")), _ptr(o["planes"]), _ptr(o["sigma"]),
                                    _ptr(o["snr"]), _ptr(o["peaks"]), _stream()))
        return o


def _fill_job(a, j):
    """Fill an AmapJob from a dict of tensors; returns the tensors used."""
    a.n = _side(j["g1"])
    a.J = int(j["planes"].shape[0])
    a.n_real = int(j.get("n_real", 0))
    a.seed = int(j.get("seed", 0))
    a.threshold = float(j.get("threshold", 3.0))
    used = []
    for key in ("g1", "g2", "kappa_e", "planes", "sigma", "snr", "peaks"):
        t = j.get(key)
        setattr(a, key, _ptr(t).value if t is not None else None)
        if t is not None:
            used.append(t)
    return used


class BatchPlan:
    """A batch of maps run as one unit (amap_batch_plan / amap_batch_run).

    ``jobs`` is a list of dicts with tensors ``g1``, ``g2``, ``planes`` and
    optionally ``kappa_e``; jobs with noise realisations also carry
    ``n_real``, ``seed``, ``threshold``, ``sigma``, ``snr`` and ``peaks``.
    The plan keeps references to the tensors; on a non-default stream the
    first run captures a graph that later runs replay.
    """

    def __init__(self, ctx, jobs):
        if not jobs:
            raise ValueError("need at least one job")
        dt = _dt(jobs[0]["g1"])
        arr = (AmapJob * len(jobs))()
        self._keep = []
        for i, j in enumerate(jobs):
            if _dt(j["g1"]) != dt:
                raise TypeError("all jobs of a plan share one dtype")
            self._keep += _fill_job(arr[i], j)
        self._jobs = arr
        h = ctypes.c_void_p()
        _check(load().amap_batch_plan(ctx._h, dt, arr, len(jobs), ctypes.byref(h)))
        self._h = h
        self._ctx = ctx

    def run(self):
        _check(load().amap_batch_run(self._h, _stream()))

    def run_on(self, stream):
        """Run on an explicit HIP stream handle (None: the null stream,
        kernels launched directly without a graph)."""
        _check(load().amap_batch_run(self._h, stream))

    def close(self):
        if self._h:
            load().amap_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching request loop (amap_server_*): jobs are admitted
    by workspace footprint against ``mem_budget`` bytes into
    ``max_inflight`` concurrent slots.  Jobs are dicts as for BatchPlan."""

    def __init__(self, ctx, dtype=torch.float32, mem_budget=8 << 30, max_inflight=4,
                 max_queued=4096):
        dt = F32 if dtype == torch.float32 else F64
        h = ctypes.c_void_p()
        _check(load().amap_server_create(ctx._h, dt, int(mem_budget), int(max_inflight),
                                         int(max_queued), ctypes.byref(h)))
        self._h = h
        self._ctx = ctx
        self._held = {}

    def submit(self, job):
        """Queue a job; it runs after the work already enqueued on torch's
        current stream.  Returns its ticket."""
        a = AmapJob()
        used = _fill_job(a, job)
        t = ctypes.c_longlong()
        _check(load().amap_server_submit(self._h, ctypes.byref(a), _stream(), ctypes.byref(t)))
        self._held[t.value] = used
        return t.value

    def poll(self, ticket):
        d = ctypes.c_int()
        _check(load().amap_server_poll(self._h, int(ticket), ctypes.byref(d)))
        if d.value:
            self._held.pop(ticket, None)
        return bool(d.value)

    def wait(self, ticket):
        _check(load().amap_server_wait(self._h, int(ticket)))
        self._held.pop(ticket, None)

    def completed(self, cap=1024):
        """Tickets finished since the last call (admits queued work first)."""
        buf = (ctypes.c_longlong * cap)()
        k = ctypes.c_int()
        _check(load().amap_server_completed(self._h, buf, cap, ctypes.byref(k)))
        done = list(buf[:k.value])
        for t in done:
            self._held.pop(t, None)
        return done

    def stats(self):
        q, f, m = ctypes.c_int(), ctypes.c_int(), ctypes.c_size_t()
        _check(load().amap_server_stats(self._h, ctypes.byref(q), ctypes.byref(f), ctypes.byref(m)))
        return {"queued": q.value, "inflight": f.value, "mem_in_use": m.value}

    def close(self):
        if self._h:
            load().amap_server_destroy(self._h)
            self._h = None
            self._held.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

