"""ctypes binding of libbg (include/bg.h): argument marshalling only.

Every step of the event path runs in the HIP kernels of libbg.so; this module only
checks torch tensors (device, dtype, contiguity, shape), builds the C structs and passes
torch's current stream.  Importing it fails loudly when libbg.so has not been built.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbg.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1002_3446_amd.build`")

_lib = ctypes.CDLL(LIB_PATH)
_lib.bg_source_hash.restype = ctypes.c_char_p
_lib.bg_source_hash.argtypes = []


def _expected_hash() -> str:
    from .build import source_hash
    return source_hash()


SOURCE_HASH = _lib.bg_source_hash().decode()
if SOURCE_HASH != _expected_hash():
    raise ImportError(f"{LIB_PATH} was built from other sources (library {SOURCE_HASH}, tree {_expected_hash()}): "
                      "rebuild it with `python -m paper_1002_3446_amd.build`")

BG_OK, BG_EINVAL, BG_ENOTSUP, BG_EHIP, BG_ENOMEM = 0, -1, -2, -3, -4


class BgConfig(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32), ("prec", ctypes.c_int32), ("sqrt_s", ctypes.c_double),
        ("use_pdf", ctypes.c_int32), ("pdf_b", ctypes.c_int32), ("pdf_a", ctypes.c_double),
        ("tau_min", ctypes.c_double), ("alpha_s", ctypes.c_double), ("pt_min", ctypes.c_double),
        ("eta_max", ctypes.c_double), ("dr_min", ctypes.c_double), ("random_order", ctypes.c_int32),
        ("polarisation", ctypes.c_int32), ("seed", ctypes.c_uint64), ("first_event", ctypes.c_uint64),
        ("dynamic_scale", ctypes.c_int32), ("reserved", ctypes.c_int32), ("mu0", ctypes.c_double),
        ("pdf_da", ctypes.c_double), ("pdf_db", ctypes.c_double),
    ]


class BgInputs(ctypes.Structure):
    _fields_ = [("uniforms", ctypes.c_void_p), ("x12", ctypes.c_void_p), ("hel", ctypes.c_void_p),
                ("order", ctypes.c_void_p)]


OUTPUT_FIELDS = ("weight", "amp2", "obs", "pass", "momenta", "hel", "order", "x12", "uniforms", "acc", "logw")


class BgOutputs(ctypes.Structure):
    _fields_ = [(f, ctypes.c_void_p) for f in OUTPUT_FIELDS]


class BgHistAxis(ctypes.Structure):
    _fields_ = [("column", ctypes.c_int32), ("nbins", ctypes.c_int32), ("lo", ctypes.c_double),
                ("hi", ctypes.c_double)]


HIST_LIMBS = 12
_i64p = ctypes.POINTER(ctypes.c_int64)
_lib.bg_generate.argtypes = [ctypes.POINTER(BgConfig), ctypes.c_int, _i64p, ctypes.POINTER(BgInputs),
                             ctypes.POINTER(BgOutputs), ctypes.c_void_p]
_lib.bg_generate_noalloc.argtypes = [ctypes.POINTER(BgConfig), ctypes.c_int64, ctypes.POINTER(BgInputs),
                                     ctypes.POINTER(BgOutputs), ctypes.c_void_p]
_lib.bg_amp2.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64] + [ctypes.c_void_p] * 5
_lib.bg_amp2_grad.argtypes = [ctypes.POINTER(BgConfig), ctypes.c_int64] + [ctypes.c_void_p] * 9
_lib.bg_check_events.argtypes = [ctypes.c_int, ctypes.c_int64] + [ctypes.c_void_p] * 4
_lib.bg_hist_accumulate.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                    ctypes.POINTER(BgHistAxis), ctypes.c_void_p, ctypes.c_void_p]
_lib.bg_hist_read.argtypes = [ctypes.c_int, ctypes.POINTER(BgHistAxis), ctypes.c_void_p, ctypes.c_void_p,
                              ctypes.c_void_p]
_lib.bg_set_launch.argtypes = [ctypes.c_int] * 4
_lib.bg_get_launch.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
_lib.bg_set_lanes.argtypes = [ctypes.c_int] * 3
_lib.bg_get_lanes.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
_lib.bg_set_form.argtypes = [ctypes.c_int] * 3
_lib.bg_get_form.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
_lib.bg_set_mixed_launch.argtypes = [ctypes.c_int]
_lib.bg_get_mixed_launch.argtypes = []
_lib.bg_strerror.restype = ctypes.c_char_p
_lib.bg_strerror.argtypes = [ctypes.c_int]
_lib.bg_fma_rate.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]
for _f in ("bg_generate", "bg_generate_noalloc", "bg_hist_accumulate", "bg_hist_read", "bg_amp2", "bg_amp2_grad", "bg_set_launch", "bg_get_launch", "bg_version",
           "bg_set_mixed_launch", "bg_get_mixed_launch", "bg_set_lanes", "bg_get_lanes", "bg_set_form",
           "bg_get_form", "bg_fma_rate"):
    getattr(_lib, _f).restype = ctypes.c_int


class BgError(RuntimeError):
    def __init__(self, fn: str, status: int):
        super().__init__(f"{fn}: {_lib.bg_strerror(status).decode()} (status {status})")
        self.status = status


def _check(fn: str, status: int):
    if status != BG_OK:
        raise BgError(fn, status)


def version() -> int:
    return _lib.bg_version()


def fma_rate(prec: int) -> float:
    """TFLOP/s of plain fused multiply-add chains in FP32 or FP64 on the current device."""
    v = ctypes.c_double()
    _check("bg_fma_rate", _lib.bg_fma_rate(prec, ctypes.byref(v), _stream(torch.device("cuda"))))
    return v.value


def source_hash() -> str:
    """Hash of the sources the loaded library was built from (equal to the tree's)."""
    return SOURCE_HASH


def strerror(status: int) -> str:
    return _lib.bg_strerror(status).decode()


def config(n: int, prec: int = 32, sqrt_s: float = 14000.0, use_pdf: int = 1, pdf_a: float = -1.3,
           pdf_b: int = 5, tau_min: float = 0.0, alpha_s: float = 0.118, pt_min: float = 20.0,
           eta_max: float = 2.5, dr_min: float = 0.4, random_order: int = 1, seed: int = 0,
           first_event: int = 0, polarisation: int = 0, dynamic_scale: int = 0, mu0: float = 91.188,
           pdf_da: float = -0.05, pdf_db: float = 0.4) -> BgConfig:
    """polarisation: 0 helicity states, 1 random real unit vectors (real currents).
    dynamic_scale: 1 evaluates alpha_s and the density at mu = H_T (grid interpolation)."""
    return BgConfig(n, prec, sqrt_s, use_pdf, pdf_b, pdf_a, tau_min, alpha_s, pt_min, eta_max, dr_min,
                    random_order, polarisation, seed, first_event, dynamic_scale, 0, mu0, pdf_da, pdf_db)


def _ptr(t, dtype, shape, name):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name}: expected a CUDA/HIP tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name}: expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: expected shape {tuple(shape)}, got {tuple(t.shape)}")
    return t.data_ptr()


def _stream(device):
    return torch.cuda.current_stream(device).cuda_stream


_OUT_SPEC = {  # name -> (dtype, shape given N and n)
    "weight": (torch.float64, lambda N, n: (N,)),
    "amp2": (torch.float64, lambda N, n: (N,)),
    "obs": (torch.float64, lambda N, n: (N, 2)),
    "pass": (torch.uint8, lambda N, n: (N,)),
    "momenta": (torch.float64, lambda N, n: (N, n, 4)),
    "hel": (torch.int32, lambda N, n: (N,)),
    "order": (torch.uint8, lambda N, n: (N, n)),
    "x12": (torch.float64, lambda N, n: (N, 2)),
    "uniforms": (torch.float64, lambda N, n: (N, 4 * (n - 2))),
    "acc": (torch.float64, lambda N, n: (4,)),
    "logw": (torch.float64, lambda N, n: (N,)),
}


def generate(cfgs, counts, inputs=None, outputs=("weight", "amp2", "obs", "pass", "acc"), device="cuda",
             out_tensors=None):
    """Runs bg_generate over one or more classes.

    cfgs: BgConfig or list of them; counts: int or list; inputs: None or (list of) dicts
    with optional 'uniforms', 'x12', 'hel' (int32 words), 'order' tensors; outputs: names
    to allocate (helicity words come back as int32 tensors holding the uint32 bits).
    Returns a list of dicts of tensors (a single dict for a single class)."""
    single = isinstance(cfgs, BgConfig)
    cfgs = [cfgs] if single else list(cfgs)
    counts = [counts] if single else list(counts)
    if inputs is not None and isinstance(inputs, dict):
        inputs = [inputs]
    k = len(cfgs)
    carr = (BgConfig * k)(*cfgs)
    narr = (ctypes.c_int64 * k)(*counts)
    outs = (BgOutputs * k)()
    ins = (BgInputs * k)() if inputs is not None else None
    results = []
    keep = []
    for j, (c, N) in enumerate(zip(cfgs, counts)):
        n = c.n
        res = {}
        for name in outputs:
            dt, sh = _OUT_SPEC[name]
            if out_tensors is not None and name in out_tensors[j]:
                t = out_tensors[j][name]
            else:
                t = torch.zeros(sh(N, n), dtype=dt, device=device)
            setattr(outs[j], name, _ptr(t, dt, sh(N, n), name))
            res[name] = t
        if ins is not None and inputs[j] is not None:
            d = inputs[j]
            ins[j].uniforms = _ptr(d.get("uniforms"), torch.float64, (N, 4 * (n - 2)), "uniforms")
            ins[j].x12 = _ptr(d.get("x12"), torch.float64, (N, 2), "x12")
            ins[j].hel = _ptr(d.get("hel"), torch.int32, (N,), "hel")
            ins[j].order = _ptr(d.get("order"), torch.uint8, (N, n), "order")
            keep.append(d)
        results.append(res)
    st = _lib.bg_generate(carr, k, narr, ins, outs, _stream(torch.device(device)))
    _check("bg_generate", st)
    return results[0] if single else results


def generate_noalloc(cfg, N, out_tensors, inputs=None, device="cuda"):
    """bg_generate_noalloc for one class into caller-allocated tensors (out_tensors: dict of
    output name -> tensor, shapes as in generate); the library allocates nothing."""
    outs = BgOutputs()
    for name, t in out_tensors.items():
        dt, sh = _OUT_SPEC[name]
        setattr(outs, name, _ptr(t, dt, sh(N, cfg.n), name))
    ins = None
    if inputs is not None:
        ins = BgInputs()
        n = cfg.n
        ins.uniforms = _ptr(inputs.get("uniforms"), torch.float64, (N, 4 * (n - 2)), "uniforms")
        ins.x12 = _ptr(inputs.get("x12"), torch.float64, (N, 2), "x12")
        ins.hel = _ptr(inputs.get("hel"), torch.int32, (N,), "hel")
        ins.order = _ptr(inputs.get("order"), torch.uint8, (N, n), "order")
    st = _lib.bg_generate_noalloc(ctypes.byref(cfg), N, ctypes.byref(ins) if ins is not None else None,
                                  ctypes.byref(outs), _stream(torch.device(device)))
    _check("bg_generate_noalloc", st)
    return out_tensors


OBS_HT, OBS_RMIN = 0, 1


def _axes(axes):
    """axes: sequence of (column, nbins, lo, hi) -> ctypes array, total bins."""
    arr = (BgHistAxis * len(axes))(*[BgHistAxis(int(c), int(nb), float(lo), float(hi)) for c, nb, lo, hi in axes])
    return arr, sum(int(a[1]) + 2 for a in axes)


def hist_limbs(axes, device="cuda"):
    """A zeroed limb array for bg_hist_accumulate over these axes."""
    _, total = _axes(axes)
    return torch.zeros((total, 2, HIST_LIMBS), dtype=torch.int64, device=device)


def hist_accumulate(weight, obs, axes, limbs):
    """Adds the events (weight [N], obs [N, 2] float64) into limbs (hist_limbs), exactly."""
    arr, total = _axes(axes)
    N = weight.shape[0]
    st = _lib.bg_hist_accumulate(N, _ptr(weight, torch.float64, (N,), "weight"), _ptr(obs, torch.float64, (N, 2), "obs"),
                                 len(axes), arr, _ptr(limbs, torch.int64, (total, 2, HIST_LIMBS), "limbs"),
                                 _stream(limbs.device))
    _check("bg_hist_accumulate", st)
    return limbs


def hist_read(axes, limbs):
    """[total bins, 2] float64: (sum w, sum w^2) per bin, underflow and overflow included, in
    axis order; each the correctly rounded exact sum."""
    arr, total = _axes(axes)
    out = torch.empty((total, 2), dtype=torch.float64, device=limbs.device)
    st = _lib.bg_hist_read(len(axes), arr, _ptr(limbs, torch.int64, (total, 2, HIST_LIMBS), "limbs"),
                           _ptr(out, torch.float64, (total, 2), "out"), _stream(limbs.device))
    _check("bg_hist_read", st)
    return out


# BG_DEBUG=1 in the environment: amp2 and amp2_grad validate their orderings and helicity
# words with bg_check_events first (one device synchronisation per call)
DEBUG_CHECKS = os.environ.get("BG_DEBUG", "") not in ("", "0")


def check_events(n: int, hel, order) -> int:
    """Index of the first event whose order row is not a permutation of 0..n-1 or whose
    helicity word has a bit at or above n; -1 when all are well formed.  Synchronises the
    current stream to read the result."""
    N = order.shape[0]
    res = torch.empty(1, dtype=torch.int64, device=order.device)
    st = _lib.bg_check_events(n, N, _ptr(hel, torch.int32, (N,), "hel"), _ptr(order, torch.uint8, (N, n), "order"),
                              _ptr(res, torch.int64, (1,), "first_bad"), _stream(order.device))
    _check("bg_check_events", st)
    return int(res.item())


def _debug_check(fn: str, n: int, hel, order):
    bad = check_events(n, hel, order)
    if bad >= 0:
        raise ValueError(f"{fn}: event {bad} has a malformed ordering or helicity word")


def amp2(n: int, prec: int, mom, hel, order, out=None):
    """|A(sigma;h)|^2 for momenta [N, n, 4] float64, hel [N] int32 words, order [N, n] uint8."""
    N = mom.shape[0]
    if DEBUG_CHECKS and N > 0:
        _debug_check("bg_amp2", n, hel, order)
    if out is None:
        out = torch.empty(N, dtype=torch.float64, device=mom.device)
    st = _lib.bg_amp2(n, prec, N, _ptr(mom, torch.float64, (N, n, 4), "mom"), _ptr(hel, torch.int32, (N,), "hel"),
                      _ptr(order, torch.uint8, (N, n), "order"), _ptr(out, torch.float64, (N,), "out"),
                      _stream(mom.device))
    _check("bg_amp2", st)
    return out


def amp2_grad(cfg: BgConfig, u, x12, hel, order, gout=None, want_logw=True):
    """(grad_u [N, 4(n-2)], grad_x [N, 2], log w_int [N]) of the log integrand weight."""
    N = u.shape[0]
    n = cfg.n
    if DEBUG_CHECKS and N > 0:
        _debug_check("bg_amp2_grad", n, hel, order)
    gu = torch.empty((N, 4 * (n - 2)), dtype=torch.float64, device=u.device)
    gx = torch.empty((N, 2), dtype=torch.float64, device=u.device)
    lw = torch.empty(N, dtype=torch.float64, device=u.device) if want_logw else None
    st = _lib.bg_amp2_grad(ctypes.byref(cfg), N, _ptr(u, torch.float64, (N, 4 * (n - 2)), "u"),
                           _ptr(x12, torch.float64, (N, 2), "x12"), _ptr(hel, torch.int32, (N,), "hel"),
                           _ptr(order, torch.uint8, (N, n), "order"), _ptr(gout, torch.float64, (N,), "gout"),
                           _ptr(gu, torch.float64, (N, 4 * (n - 2)), "grad_u"),
                           _ptr(gx, torch.float64, (N, 2), "grad_x"),
                           _ptr(lw, torch.float64, (N,), "logw") if lw is not None else None,
                           _stream(u.device))
    _check("bg_amp2_grad", st)
    return gu, gx, lw


def set_launch(n: int, prec: int, block: int, tile_iters: int):
    """Threads per workgroup and events per lane in a multi-class tile; (0, 0) = default."""
    _check("bg_set_launch", _lib.bg_set_launch(n, prec, block, tile_iters))


def get_launch(n: int, prec: int):
    b, c = ctypes.c_int(), ctypes.c_int()
    _check("bg_get_launch", _lib.bg_get_launch(n, prec, ctypes.byref(b), ctypes.byref(c)))
    return b.value, c.value


def set_lanes(n: int, prec: int, lanes: int):
    """Lanes per event of the single-class kernels of (n, prec): 1, 2, 4 or 0 (default)."""
    _check("bg_set_lanes", _lib.bg_set_lanes(n, prec, lanes))


def get_lanes(n: int, prec: int) -> int:
    v = ctypes.c_int()
    _check("bg_get_lanes", _lib.bg_get_lanes(n, prec, ctypes.byref(v)))
    return v.value


FORM_DIRECT, FORM_WTENSOR = 0, 1


def set_form(n: int, prec: int, form: int):
    """Recursion form of the single-class kernels of (n, prec): FORM_DIRECT or FORM_WTENSOR."""
    _check("bg_set_form", _lib.bg_set_form(n, prec, form))


def get_form(n: int, prec: int) -> int:
    v = ctypes.c_int()
    _check("bg_get_form", _lib.bg_get_form(n, prec, ctypes.byref(v)))
    return v.value


MIXED_SEQUENTIAL, MIXED_PERSISTENT, MIXED_CONCURRENT = 0, 1, 2


def set_mixed_launch(mode: int):
    """Strategy for calls with several classes: MIXED_SEQUENTIAL (one class after another),
    MIXED_PERSISTENT (FP32 classes in one persistent launch) or MIXED_CONCURRENT (classes
    on concurrent side streams)."""
    _check("bg_set_mixed_launch", _lib.bg_set_mixed_launch(int(mode)))


def get_mixed_launch() -> int:
    return int(_lib.bg_get_mixed_launch())


TUNING_PATH = os.path.join(_HERE, "autotune.json")


def load_tuning(path: str = TUNING_PATH) -> int:
    """Applies launch shapes written by paper_1002_3446_amd.autotune; returns how many."""
    import json
    if not os.path.exists(path):
        return 0
    doc = json.load(open(path))
    entries = doc.get("shapes", [])
    for e in entries:
        set_launch(int(e["n"]), int(e["prec"]), int(e["block"]), int(e["tile_iters"]))
        if "lanes" in e:
            set_lanes(int(e["n"]), int(e["prec"]), int(e["lanes"]))
        if "form" in e:
            set_form(int(e["n"]), int(e["prec"]), int(e["form"]))
    if "mixed_mode" in doc:
        set_mixed_launch(int(doc["mixed_mode"]))
    return len(entries)


load_tuning()


def raw():
    """The loaded ctypes library (for ABI tests)."""
    return _lib
