"""ctypes binding of libtn3d.so (declarations in include/tn3d.h).

Argument marshalling only: device buffers are torch CUDA tensors whose
data_ptr() is handed to the library, and the stream is torch's current HIP
stream.  Every computation runs in the library's HIP kernels; if the library
is missing this module raises instead of computing anything itself.
"""

from __future__ import annotations

import ctypes
import weakref
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtn3d.so")

PREC_FP64 = 0
PREC_FP32 = 1
PREC_BF16 = 2
FLAG_NUMERIC = 1
FLAG_TRUNC_CLUSTER = 2
FLAG_NEAR_TIE = 4
FLAG_NO_CONVERGE = 8
FLAG_RESWEPT = 16
FLAG_INCONSISTENT = 32
OPT_GRAM_FACTOR = 1

STATUS = {0: "OK", -1: "INVALID", -2: "INCONSISTENT", -3: "UNSUPPORTED", -4: "OOM", -5: "DEVICE",
          -6: "NUMERIC"}

# every entry point declared in include/tn3d.h
SYMBOLS = [
    "tn3d_params_default", "tn3d_ctx_create", "tn3d_ctx_destroy", "tn3d_last_error",
    "tn3d_net_surface3d_point", "tn3d_net_rotated_phenom", "tn3d_net_surface3d_depolarizing",
    "tn3d_net_surface3d_loop", "tn3d_net_surface3d_wht", "tn3d_net_from_dem", "tn3d_net_num_detectors",
    "tn3d_net_num_mechanisms", "tn3d_net_num_cosets", "tn3d_net_shape", "tn3d_net_destroy",
    "tn3d_contract_cosets", "tn3d_contract_cosets_noalloc", "tn3d_decode", "tn3d_ctx_set_timing",
    "tn3d_last_timing", "tn3d_last_stats", "tn3d_autotune",
    "tn3d_ctx_set_graphs", "tn3d_ctx_graphs_cached", "tn3d_grad_loglik", "tn3d_net_from_layers",
    "tn3d_net_with_gauge_rounds",
]


MAX_CHI_LAYERS = 32


class Params(ctypes.Structure):
    _fields_ = [
        ("chi", ctypes.c_int32), ("chi_mps", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("reserved0", ctypes.c_int32), ("eps_rel", ctypes.c_double), ("tau_gap", ctypes.c_double),
        ("near_tie", ctypes.c_double), ("workspace_bytes", ctypes.c_int64), ("flags", ctypes.c_uint32),
        ("reserved1", ctypes.c_uint32), ("n_chi_layers", ctypes.c_int32),
        ("chi_layers", ctypes.c_int32 * MAX_CHI_LAYERS),
    ]

    def set_chi_schedule(self, chis):
        """Per-layer truncation caps (layer l uses chis[min(l, len - 1)]);
        an empty sequence restores the constant chi."""
        chis = [int(v) for v in chis]
        if len(chis) > MAX_CHI_LAYERS:
            raise ValueError(f"at most {MAX_CHI_LAYERS} entries")
        self.n_chi_layers = len(chis)
        for i, v in enumerate(chis):
            self.chi_layers[i] = v


_lib = None


def load_library(path: str | None = None):
    """Load libtn3d.so (built by paper_2310_10722_amd.build)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is missing: build it with paper_2310_10722_amd.build.build()")
    lib = ctypes.CDLL(p)
    c_p, i32, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    lib.tn3d_params_default.argtypes = [ctypes.POINTER(Params), i32, i32, i32]
    lib.tn3d_params_default.restype = None
    lib.tn3d_ctx_create.argtypes = [i32, c_p, ctypes.POINTER(c_p)]
    lib.tn3d_ctx_destroy.argtypes = [c_p]
    lib.tn3d_ctx_destroy.restype = None
    lib.tn3d_last_error.argtypes = [c_p]
    lib.tn3d_last_error.restype = ctypes.c_char_p
    lib.tn3d_net_surface3d_point.argtypes = [c_p, i32, ctypes.POINTER(f64), ctypes.POINTER(c_p)]
    lib.tn3d_net_rotated_phenom.argtypes = [c_p, i32, i32, ctypes.POINTER(f64), ctypes.POINTER(c_p)]
    lib.tn3d_net_surface3d_depolarizing.argtypes = [c_p, i32, ctypes.POINTER(f64), ctypes.POINTER(c_p)]
    lib.tn3d_net_surface3d_loop.argtypes = [c_p, i32, ctypes.POINTER(f64), ctypes.POINTER(c_p)]
    lib.tn3d_net_surface3d_wht.argtypes = [c_p, i32, i32, ctypes.POINTER(f64), ctypes.POINTER(c_p)]
    lib.tn3d_net_from_dem.argtypes = [c_p, i32, i32, ctypes.c_int64, c_p, c_p, ctypes.POINTER(f64), i32, c_p, c_p,
                                      ctypes.POINTER(c_p)]
    for f in ("tn3d_net_num_detectors", "tn3d_net_num_mechanisms", "tn3d_net_num_cosets"):
        getattr(lib, f).argtypes = [c_p]
        getattr(lib, f).restype = i32
    lib.tn3d_net_shape.argtypes = [c_p, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.tn3d_net_shape.restype = None
    lib.tn3d_net_destroy.argtypes = [c_p]
    lib.tn3d_net_destroy.restype = None
    lib.tn3d_contract_cosets.argtypes = [c_p, i32, ctypes.POINTER(c_p), c_p, c_p, ctypes.POINTER(Params), c_p,
                                         c_p]
    lib.tn3d_contract_cosets_noalloc.argtypes = lib.tn3d_contract_cosets.argtypes
    lib.tn3d_decode.argtypes = [c_p, i32, ctypes.POINTER(c_p), c_p, c_p, ctypes.POINTER(Params), c_p, c_p, c_p,
                                c_p]
    lib.tn3d_ctx_set_timing.argtypes = [c_p, i32]
    lib.tn3d_ctx_set_graphs.argtypes = [c_p, i32]
    lib.tn3d_ctx_graphs_cached.argtypes = [c_p]
    lib.tn3d_ctx_graphs_cached.restype = i32
    lib.tn3d_last_timing.argtypes = [c_p, ctypes.POINTER(f64), i32]
    lib.tn3d_last_stats.argtypes = [c_p, ctypes.POINTER(f64), i32]
    lib.tn3d_autotune.argtypes = [c_p, i32, ctypes.POINTER(c_p), c_p, c_p, ctypes.POINTER(Params),
                                  ctypes.POINTER(f64), i32]
    lib.tn3d_autotune.restype = i32
    lib.tn3d_grad_loglik.argtypes = [c_p, c_p, i32, c_p, c_p, ctypes.POINTER(Params), i32, c_p, c_p, c_p, c_p, c_p,
                                     c_p]
    lib.tn3d_grad_loglik.restype = i32
    lib.tn3d_net_from_layers.argtypes = [c_p, i32, i32, i32, i32, i32, c_p, c_p, i32, c_p, c_p, c_p,
                                         ctypes.c_int64, ctypes.c_double, ctypes.POINTER(c_p)]
    lib.tn3d_net_from_layers.restype = i32
    lib.tn3d_net_with_gauge_rounds.argtypes = [c_p, c_p, i32, ctypes.POINTER(c_p)]
    lib.tn3d_net_with_gauge_rounds.restype = i32
    lib.tn3d_last_stats.restype = i32
    for f in ("tn3d_ctx_create", "tn3d_net_surface3d_point", "tn3d_net_rotated_phenom",
              "tn3d_net_surface3d_depolarizing", "tn3d_net_surface3d_loop", "tn3d_net_surface3d_wht", "tn3d_net_from_dem", "tn3d_contract_cosets", "tn3d_contract_cosets_noalloc",
              "tn3d_decode", "tn3d_ctx_set_timing", "tn3d_last_timing", "tn3d_ctx_set_graphs"):
        getattr(lib, f).restype = i32
    if path is None:
        _lib = lib
    return lib


def exported_symbols(path: str | None = None):
    """Names from SYMBOLS that the library exports (no device call is made)."""
    lib = ctypes.CDLL(path or LIB_PATH)
    out = []
    for s in SYMBOLS:
        try:
            getattr(lib, s)
            out.append(s)
        except AttributeError:
            pass
    return out


class Tn3dError(RuntimeError):
    pass


def _check(lib, ctx, st):
    if st != 0:
        msg = lib.tn3d_last_error(ctx).decode() if ctx else ""
        raise Tn3dError(f"tn3d status {STATUS.get(st, st)}: {msg}")


def tn3d_params_default(chi: int, chi_mps: int | None = None, precision: int = PREC_FP32) -> Params:
    p = Params()
    load_library().tn3d_params_default(ctypes.byref(p), chi, chi if chi_mps is None else chi_mps, precision)
    return p


class Context:
    """tn3d_ctx on a torch CUDA device, enqueueing on torch's current stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.lib = load_library()
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self._stream = stream
        h = ctypes.c_void_p()
        _check(self.lib, None, self.lib.tn3d_ctx_create(device, ctypes.c_void_p(stream.cuda_stream),
                                                        ctypes.byref(h)))
        self.h = h
        self._nets = weakref.WeakSet()

    def close(self):
        if self.h:
            # the networks of this context go first (the library's contract)
            for net in list(self._nets):
                net.close()
            self.lib.tn3d_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_timing(self, level=True):
        """0/False off, 1/True kernel times, 2 times and bond statistics."""
        _check(self.lib, self.h, self.lib.tn3d_ctx_set_timing(self.h, int(level)))

    def set_graphs(self, on: bool = True):
        _check(self.lib, self.h, self.lib.tn3d_ctx_set_graphs(self.h, 1 if on else 0))

    def graphs_cached(self) -> int:
        return int(self.lib.tn3d_ctx_graphs_cached(self.h))

    def last_timing(self):
        out = (ctypes.c_double * 15)()
        _check(self.lib, self.h, self.lib.tn3d_last_timing(self.h, out, 15))
        return list(out)

    def last_stats(self):
        out = (ctypes.c_double * 7)()
        _check(self.lib, self.h, self.lib.tn3d_last_stats(self.h, out, 7))
        return list(out)


class Net:
    """A network handle built by one of the family builders."""

    def __init__(self, ctx: Context, h):
        self.ctx = ctx
        self.h = h
        ctx._nets.add(self)
        lib = ctx.lib
        self.n_det = lib.tn3d_net_num_detectors(h)
        self.n_mech = lib.tn3d_net_num_mechanisms(h)
        self.n_cosets = lib.tn3d_net_num_cosets(h)
        a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        lib.tn3d_net_shape(h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
        self.shape = (a.value, b.value, c.value)

    def close(self):
        if self.h:
            # after its context was closed the handle is detached and only
            # freed (the library released its device arrays then)
            self.ctx.lib.tn3d_net_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _rates(p, n):
    """The rate array as contiguous float64 of exactly n entries (the
    builders read n values through the pointer)."""
    a = np.ascontiguousarray(np.asarray(p, dtype=np.float64)).reshape(-1)
    if a.size != n:
        raise ValueError(f"expected {n} rates, got {a.size}")
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _n_cubic(L):
    return L ** 3 + 2 * L * (L - 1) ** 2 if L >= 2 else 0


def tn3d_net_surface3d_point(ctx: Context, L: int, p_mech) -> Net:
    a, ptr = _rates(p_mech, _n_cubic(L)) if L >= 2 else _rates(np.zeros(1), 1)
    h = ctypes.c_void_p()
    _check(ctx.lib, ctx.h, ctx.lib.tn3d_net_surface3d_point(ctx.h, L, ptr, ctypes.byref(h)))
    return Net(ctx, h)


def tn3d_net_rotated_phenom(ctx: Context, d: int, T: int, p_mech) -> Net:
    ok = d >= 3 and d % 2 == 1 and T >= 1
    a, ptr = _rates(p_mech, T * d * d + T * (d * d - 1) // 2) if ok else _rates(np.zeros(1), 1)
    h = ctypes.c_void_p()
    _check(ctx.lib, ctx.h, ctx.lib.tn3d_net_rotated_phenom(ctx.h, d, T, ptr, ctypes.byref(h)))
    return Net(ctx, h)


def tn3d_net_surface3d_depolarizing(ctx: Context, L: int, p_qubit) -> Net:
    a, ptr = _rates(p_qubit, _n_cubic(L)) if L >= 2 else _rates(np.zeros(1), 1)
    h = ctypes.c_void_p()
    _check(ctx.lib, ctx.h, ctx.lib.tn3d_net_surface3d_depolarizing(ctx.h, L, ptr, ctypes.byref(h)))
    return Net(ctx, h)


def tn3d_net_surface3d_loop(ctx: Context, L: int, p_mech) -> Net:
    a, ptr = _rates(p_mech, _n_cubic(L)) if L >= 2 else _rates(np.zeros(1), 1)
    h = ctypes.c_void_p()
    _check(ctx.lib, ctx.h, ctx.lib.tn3d_net_surface3d_loop(ctx.h, L, ptr, ctypes.byref(h)))
    return Net(ctx, h)


def tn3d_net_from_dem(ctx: Context, H, p_mech, obs, det_coord) -> Net:
    """H: dense 0/1 [n_det, n_mech] (passed as its COO pattern), p_mech
    [n_mech], obs [n_mech] (one observable row), det_coord [n_det, 3] ints."""
    H = np.asarray(H, dtype=np.uint8)
    n_det, n_mech = H.shape
    d_idx, m_idx = np.nonzero(H & 1)
    d_idx = np.ascontiguousarray(d_idx, dtype=np.int32)
    m_idx = np.ascontiguousarray(m_idx, dtype=np.int32)
    a, ptr = _rates(p_mech, n_mech)
    ob = np.ascontiguousarray(np.asarray(obs, dtype=np.uint8).reshape(-1))
    if ob.size != n_mech:
        raise ValueError(f"expected {n_mech} observable entries, got {ob.size}")
    co = np.ascontiguousarray(np.asarray(det_coord, dtype=np.int32).reshape(-1))
    if co.size != 3 * n_det:
        raise ValueError(f"expected {3 * n_det} coordinates, got {co.size}")
    h = ctypes.c_void_p()
    _check(ctx.lib, ctx.h, ctx.lib.tn3d_net_from_dem(ctx.h, n_det, n_mech, d_idx.size, d_idx.ctypes.data,
                                                     m_idx.ctypes.data, ptr, 1, ob.ctypes.data, co.ctypes.data,
                                                     ctypes.byref(h)))
    return Net(ctx, h)


SECTOR_POINT, SECTOR_LOOP = 0, 1
OP_PRE, OP_GATE_H, OP_GATE_V, OP_POST = 0, 1, 2, 3


def tn3d_net_with_gauge_rounds(ctx: Context, base: Net, rounds: int) -> Net:
    """`base` with `rounds` rounds of identity gates on every bond before each
    layer after the first."""
    h = ctypes.c_void_p()
    _check(ctx.lib, ctx.h, ctx.lib.tn3d_net_with_gauge_rounds(ctx.h, base.h, int(rounds), ctypes.byref(h)))
    return Net(ctx, h)


class LayerOp(ctypes.Structure):
    _fields_ = [("layer", ctypes.c_int32), ("kind", ctypes.c_int32), ("x", ctypes.c_int32), ("y", ctypes.c_int32),
                ("d_in", ctypes.c_int32), ("d_out", ctypes.c_int32), ("det", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("off0", ctypes.c_int64), ("off1", ctypes.c_int64)]


def tn3d_net_from_layers(ctx: Context, lx: int, ly: int, n_layers: int, n_det: int, init_dims, init_off, ops,
                         final_off, values, split_tol: float = 1e-14) -> Net:
    """A generic layered network.  init_dims int [n_cosets, lx*ly, 5],
    init_off int [n_cosets, lx*ly], ops: sequence of (layer, kind, x, y, d_in,
    d_out, det, off0, off1), final_off int [lx*ly], values float64 (the
    tensors and matrices the offsets point into)."""
    dims = np.ascontiguousarray(np.asarray(init_dims, dtype=np.int32))
    if dims.ndim != 3 or dims.shape[1:] != (lx * ly, 5):
        raise ValueError("init_dims must have shape [n_cosets, lx * ly, 5]")
    ioff = np.ascontiguousarray(np.asarray(init_off, dtype=np.int64))
    if ioff.shape != dims.shape[:2]:
        raise ValueError("init_off must have shape [n_cosets, lx * ly]")
    foff = np.ascontiguousarray(np.asarray(final_off, dtype=np.int64).reshape(-1))
    if foff.size != lx * ly:
        raise ValueError("final_off needs lx * ly entries")
    vals = np.ascontiguousarray(np.asarray(values, dtype=np.float64).reshape(-1))
    arr = (LayerOp * max(len(ops), 1))()
    for i, o in enumerate(ops):
        layer, kind, x, y, d_in, d_out, det, off0, off1 = o
        arr[i] = LayerOp(layer, kind, x, y, d_in, d_out, det, 0, off0, off1)
    h = ctypes.c_void_p()
    _check(ctx.lib, ctx.h, ctx.lib.tn3d_net_from_layers(
        ctx.h, lx, ly, n_layers, n_det, dims.shape[0], dims.ctypes.data, ioff.ctypes.data, len(ops),
        ctypes.cast(arr, ctypes.c_void_p),
        foff.ctypes.data, vals.ctypes.data, vals.size, float(split_tol), ctypes.byref(h)))
    return Net(ctx, h)


def tn3d_net_surface3d_wht(ctx: Context, L: int, sector: int, p_mech) -> Net:
    a, ptr = _rates(p_mech, _n_cubic(L)) if L >= 2 else _rates(np.zeros(1), 1)
    h = ctypes.c_void_p()
    _check(ctx.lib, ctx.h, ctx.lib.tn3d_net_surface3d_wht(ctx.h, L, sector, ptr, ctypes.byref(h)))
    return Net(ctx, h)


def _batch_args(nets, syndromes):
    import torch
    if syndromes.dtype != torch.uint8 or not syndromes.is_cuda or syndromes.dim() != 2:
        raise ValueError("syndromes: uint8 CUDA tensor [batch, n_det]")
    syndromes = syndromes.contiguous()
    B = syndromes.shape[0]
    if isinstance(nets, Net):
        nets = [nets] * B
    if len(nets) != B:
        raise ValueError("one network per syndrome")
    if B > 0 and syndromes.shape[1] < max(n.n_det for n in nets):
        raise ValueError("syndrome rows are narrower than a network's detector count")
    offs = torch.arange(B, dtype=torch.int64, device=syndromes.device) * syndromes.shape[1]
    arr = (ctypes.c_void_p * max(B, 1))(*[n.h.value for n in nets])
    return nets, syndromes, offs, arr, B


def tn3d_contract_cosets(ctx: Context, nets, syndromes, params: Params):
    """log p_{m,L} [batch, 4] (float64 CUDA) and flags [batch] (int32 view of uint32)."""
    import torch
    nets, syn, offs, arr, B = _batch_args(nets, syndromes)
    logp = torch.empty((B, 4), dtype=torch.float64, device=syn.device)
    flags = torch.zeros((B,), dtype=torch.int32, device=syn.device)
    st = ctx.lib.tn3d_contract_cosets(ctx.h, B, arr, ctypes.c_void_p(syn.data_ptr()),
                                      ctypes.c_void_p(offs.data_ptr()), ctypes.byref(params),
                                      ctypes.c_void_p(logp.data_ptr()), ctypes.c_void_p(flags.data_ptr()))
    _check(ctx.lib, ctx.h, st)
    return logp, flags


def tn3d_autotune(ctx: Context, nets, syndromes, params: Params):
    """Chooses and caches the fastest launch shape for these networks and
    parameters; returns (index, team, mid, narrow, best ms, default ms)."""
    nets, syn, offs, arr, B = _batch_args(nets, syndromes)
    out = (ctypes.c_double * 6)()
    st = ctx.lib.tn3d_autotune(ctx.h, B, arr, ctypes.c_void_p(syn.data_ptr()), ctypes.c_void_p(offs.data_ptr()),
                               ctypes.byref(params), out, 6)
    _check(ctx.lib, ctx.h, st)
    return tuple(out)


def tn3d_contract_cosets_noalloc(ctx: Context, nets, syndromes, params: Params, logp=None, flags=None):
    """As tn3d_contract_cosets, on the library's static device scratch (no
    device allocation inside the call); logp [batch, 4] float64 and flags
    [batch] int32 CUDA tensors may be passed in, else they are made here."""
    import torch
    nets, syn, offs, arr, B = _batch_args(nets, syndromes)
    if logp is None:
        logp = torch.empty((B, 4), dtype=torch.float64, device=syn.device)
    if flags is None:
        flags = torch.zeros((B,), dtype=torch.int32, device=syn.device)
    st = ctx.lib.tn3d_contract_cosets_noalloc(ctx.h, B, arr, ctypes.c_void_p(syn.data_ptr()),
                                              ctypes.c_void_p(offs.data_ptr()), ctypes.byref(params),
                                              ctypes.c_void_p(logp.data_ptr()), ctypes.c_void_p(flags.data_ptr()))
    _check(ctx.lib, ctx.h, st)
    return logp, flags


def tn3d_decode(ctx: Context, nets, syndromes, params: Params):
    """(coset int32 [B], logratio float64 [B], logp float64 [B,4], flags int32 [B])."""
    import torch
    nets, syn, offs, arr, B = _batch_args(nets, syndromes)
    dev = syn.device
    coset = torch.empty((B,), dtype=torch.int32, device=dev)
    lr = torch.empty((B,), dtype=torch.float64, device=dev)
    logp = torch.empty((B, 4), dtype=torch.float64, device=dev)
    flags = torch.zeros((B,), dtype=torch.int32, device=dev)
    st = ctx.lib.tn3d_decode(ctx.h, B, arr, ctypes.c_void_p(syn.data_ptr()), ctypes.c_void_p(offs.data_ptr()),
                             ctypes.byref(params), ctypes.c_void_p(coset.data_ptr()),
                             ctypes.c_void_p(lr.data_ptr()), ctypes.c_void_p(logp.data_ptr()),
                             ctypes.c_void_p(flags.data_ptr()))
    _check(ctx.lib, ctx.h, st)
    return coset, lr, logp, flags


def tn3d_grad_loglik(ctx: Context, net: Net, syndromes, params: Params, rate_of_mech=None, n_rates=None,
                     per_item=False):
    """Gradient of sum_s log P(m_s) with respect to the rates (one network for
    the whole batch).  rate_of_mech: optional int array [n_mech] mapping each
    builder rate to one of n_rates parameters.  Returns (grad float64
    [n_rates], loglik_sum float64 [1], loglik float64 [B], flags int32 [B],
    grad_items float64 [B, n_mech] or None) as CUDA tensors."""
    import torch
    if not isinstance(net, Net):
        raise ValueError("one network for the batch")
    _, syn, offs, _, B = _batch_args(net, syndromes)
    dev = syn.device
    if rate_of_mech is None:
        n_rates = net.n_mech if n_rates is None else int(n_rates)
        rmap = None
    else:
        rmap = np.ascontiguousarray(np.asarray(rate_of_mech, dtype=np.int32)).reshape(-1)
        if rmap.size != net.n_mech:
            raise ValueError(f"rate_of_mech needs {net.n_mech} entries, got {rmap.size}")
        n_rates = int(rmap.max()) + 1 if n_rates is None else int(n_rates)
    grad = torch.empty((max(n_rates, 1),), dtype=torch.float64, device=dev)[:n_rates]
    total = torch.empty((1,), dtype=torch.float64, device=dev)
    loglik = torch.empty((B,), dtype=torch.float64, device=dev)
    flags = torch.zeros((B,), dtype=torch.int32, device=dev)
    items = torch.empty((B, net.n_mech), dtype=torch.float64, device=dev) if per_item else None
    st = ctx.lib.tn3d_grad_loglik(
        ctx.h, net.h, B, ctypes.c_void_p(syn.data_ptr()), ctypes.c_void_p(offs.data_ptr()), ctypes.byref(params),
        n_rates, None if rmap is None else rmap.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(grad.data_ptr()),
        ctypes.c_void_p(total.data_ptr()), ctypes.c_void_p(loglik.data_ptr()),
        None if items is None else ctypes.c_void_p(items.data_ptr()), ctypes.c_void_p(flags.data_ptr()))
    _check(ctx.lib, ctx.h, st)
    return grad, total, loglik, flags, items


def _autograd_function():
    import torch

    class LogLikelihood(torch.autograd.Function):
        """sum_s log P(m_s) as a function of the rate parameters; the
        gradient comes from tn3d_grad_loglik."""

        @staticmethod
        def forward(fctx, rates, ctx, build, syndromes, params, rate_of_mech):
            r = rates.detach().to("cpu", torch.float64).numpy()
            p_mech = r if rate_of_mech is None else r[np.asarray(rate_of_mech)]
            net = build(ctx, p_mech)
            try:
                grad, total, _, _, _ = tn3d_grad_loglik(ctx, net, syndromes, params, rate_of_mech, r.size)
            finally:
                net.close()
            fctx.save_for_backward(grad)
            return total.reshape(()).to(rates.device, rates.dtype)

        @staticmethod
        def backward(fctx, g_out):
            (grad,) = fctx.saved_tensors
            return (g_out.to(grad.device, grad.dtype) * grad).to(g_out.device, g_out.dtype), \
                None, None, None, None, None

    return LogLikelihood


def log_likelihood(ctx: Context, build, rates, syndromes, params: Params, rate_of_mech=None):
    """Differentiable sum_s log P(m_s): `rates` a float64 tensor of rate
    parameters, build(ctx, p_mech) -> Net a family builder at per-mechanism
    rates p_mech = rates[rate_of_mech] (or rates itself), syndromes a uint8
    CUDA tensor [B, n_det].  backward() fills rates.grad through
    tn3d_grad_loglik."""
    return _autograd_function().apply(rates, ctx, build, syndromes, params, rate_of_mech)


# short aliases
contract_cosets = tn3d_contract_cosets
decode = tn3d_decode
