"""MI355X (gfx950) hot path of the DISCOVER / SISSO-style symbolic regression
method (arXiv 2602.06986): candidate generation with unit pruning, SIS
screening with exact top-k, exhaustive L0 and OMP.

This module only marshals arguments to the C ABI of ``libdiscover.so``
(include/discover.h); every step of the path runs in the library's HIP
kernels.  PyTorch supplies device memory and the stream.  There is no CPU
fallback: a missing library or GPU raises.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdiscover.so")

OPS = ("exp", "log", "sqrt", "sq", "inv", "add", "sub", "mul", "div", "rdiv")
OP_BIT = {name: 1 << i for i, name in enumerate(OPS)}
SCORE_PER_TARGET, SCORE_MAX = 0, 1
FP64, BF16_GUARD, FP16_GUARD = 0, 1, 2
STATUS = {0: "OK", -1: "E_ARG", -2: "E_NOMEM", -3: "E_HIP", -4: "E_UNSUPPORTED",
          -5: "E_NUMERIC", -6: "E_CAPACITY"}


class DiscoverError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (STATUS.get(code, "?"), code, msg))
        self.code = code


class Problem(C.Structure):
    _fields_ = [("n", C.c_int32), ("p", C.c_int32), ("T", C.c_int32), ("B", C.c_int32),
                ("X", C.c_void_p), ("ldx", C.c_int64), ("Y", C.c_void_p), ("ldy", C.c_int64),
                ("units", C.c_void_p), ("exclude", C.c_void_p), ("n_exclude", C.c_int32)]


class ScreenParams(C.Structure):
    _fields_ = [("ops", C.c_uint32), ("rung", C.c_int32), ("rung_ops", C.c_uint32 * 4),
                ("rung_pool", C.c_int32 * 4), ("k", C.c_int32), ("score_mode", C.c_int32),
                ("precision", C.c_int32), ("dedup", C.c_int32), ("tile_j", C.c_int32),
                ("lp_pairs", C.c_int32), ("sched", C.c_int32)]


class ScreenStats(C.Structure):
    _fields_ = [("n_raw", C.c_int64), ("n_unit_valid", C.c_int64), ("n_scored", C.c_int64),
                ("pool_size", C.c_int64), ("pool_rounds", C.c_int64), ("n_merged", C.c_int64),
                ("n_selected", C.c_int64), ("max_lowprec_err", C.c_double),
                ("guard_band", C.c_double), ("tile_j", C.c_int32), ("status", C.c_int32)]

    def asdict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class L0Problem(C.Structure):
    _fields_ = [("n", C.c_int32), ("S", C.c_int32), ("F", C.c_void_p), ("ldf", C.c_int64),
                ("ids", C.c_void_p), ("y", C.c_void_p)]


class L0Stats(C.Structure):
    _fields_ = [("n_subsets", C.c_int64), ("n_band", C.c_int64), ("n_singular", C.c_int64),
                ("status", C.c_int32), ("reserved", C.c_int32)]

    def asdict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class AnnealParams(C.Structure):
    _fields_ = [("chains", C.c_int32), ("reserved", C.c_int32), ("steps", C.c_int64),
                ("T0", C.c_double), ("alpha", C.c_double), ("seed", C.c_uint64)]


class BnbParams(C.Structure):
    _fields_ = [("max_nodes", C.c_int64), ("reserved", C.c_int64)]


class BnbStats(C.Structure):
    _fields_ = [("n_subsets", C.c_int64), ("n_nodes", C.c_int64), ("n_bounds", C.c_int64),
                ("n_leaves", C.c_int64), ("n_refit", C.c_int64), ("m0", C.c_int32), ("status", C.c_int32)]

    def asdict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Rules(C.Structure):
    _fields_ = [("max_complexity", C.c_int32), ("forbid_nest", C.c_uint32 * 10),
                ("n_forbid_pairs", C.c_int32), ("forbid_pairs", C.c_void_p),
                ("target_unit", C.c_int32), ("target_units", C.c_int32 * 8)]


# Every symbol include/discover.h declares.
SYMBOLS = ("discover_create", "discover_destroy", "discover_last_error",
           "discover_generate_screen", "discover_l0_fit", "discover_omp", "discover_count",
           "discover_decode", "discover_set_timing", "discover_timing", "discover_reset_timing",
           "discover_sisso_batch", "discover_set_graph_timing", "discover_set_fixup_capacity",
           "discover_reserve", "discover_omp_noalloc", "discover_l0_anneal", "discover_set_rules", "discover_l0_bnb")

_lib = None


def lib():
    """Load libdiscover.so (built in-tree by paper_2602_06986_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libdiscover.so is not built; run python -m paper_2602_06986_amd.build")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.discover_create.argtypes = [C.c_int, C.POINTER(P)]
        L.discover_destroy.argtypes = [P]
        L.discover_destroy.restype = None
        L.discover_last_error.restype = C.c_char_p
        # stats: host structures (byref / arrays) or a device address
        L.discover_generate_screen.argtypes = [P, C.POINTER(Problem), C.c_int32,
                                               C.POINTER(ScreenParams), P, P, P, C.c_int64, P, P]
        L.discover_l0_fit.argtypes = [P, C.POINTER(L0Problem), C.c_int32, C.c_int32, C.c_int32,
                                      P, P, P, P, C.c_int64, P, P]
        L.discover_reserve.argtypes = [P, C.POINTER(Problem), C.c_int32, C.POINTER(ScreenParams),
                                       C.c_int32, C.c_int32, P]
        L.discover_omp.argtypes = [P, C.POINTER(L0Problem), C.c_int32, C.c_int32, P, C.c_int32,
                                   P, P, P, P, C.c_int64, P]
        L.discover_omp_noalloc.argtypes = L.discover_omp.argtypes
        L.discover_l0_anneal.argtypes = [P, C.POINTER(L0Problem), C.c_int32, C.c_int32,
                                         C.POINTER(AnnealParams), P, P, P, P, P, P, P, P, C.c_int64, P]
        L.discover_l0_bnb.argtypes = [P, C.POINTER(L0Problem), C.c_int32, C.c_int32, C.c_int32,
                                      C.POINTER(BnbParams), P, P, P, P, C.c_int64, P, P]
        L.discover_count.argtypes = [C.c_int32, C.POINTER(ScreenParams)]
        L.discover_count.restype = C.c_int64
        L.discover_decode.argtypes = [C.c_int32, C.POINTER(ScreenParams), C.c_int64, C.c_char_p,
                                      C.c_size_t]
        L.discover_set_timing.argtypes = [P, C.c_int32]
        L.discover_timing.argtypes = [P, C.c_char_p, C.POINTER(C.c_int64), C.POINTER(C.c_double)]
        L.discover_reset_timing.argtypes = [P]
        L.discover_sisso_batch.argtypes = [P, C.POINTER(Problem), C.c_int32, C.POINTER(ScreenParams),
                                           C.c_int32, C.c_int32, C.c_int32, P, P, P, P, P,
                                           C.c_int32, P, P, P, C.POINTER(C.c_int32), P]
        L.discover_set_graph_timing.argtypes = [P, C.c_char_p]
        L.discover_set_fixup_capacity.argtypes = [P, C.c_int64]
        L.discover_set_rules.argtypes = [P, C.POINTER(Rules)]
        _lib = L
    return _lib


def _check(code):
    if code != 0:
        raise DiscoverError(code, lib().discover_last_error().decode())


def params(ops=OPS, rung=1, k=20, score_mode=SCORE_PER_TARGET, precision=FP64, dedup=True,
           rung_ops=None, rung_pool=None, tile_j=0, lp_pairs=0, sched=0):
    """Build the screening parameter struct from operator names."""
    prm = ScreenParams()
    prm.ops = sum(OP_BIT[o] for o in ops)
    prm.rung = rung
    for r in range(4):
        ro = rung_ops[r] if rung_ops is not None and r < len(rung_ops) else None
        prm.rung_ops[r] = 0 if ro is None else sum(OP_BIT[o] for o in ro)
        rp = rung_pool[r] if rung_pool is not None and r < len(rung_pool) else None
        prm.rung_pool[r] = -1 if rp is None else int(rp)
    prm.k = k
    prm.score_mode = score_mode
    prm.precision = precision
    prm.dedup = 1 if dedup else 0
    prm.tile_j = tile_j
    prm.lp_pairs = lp_pairs
    prm.sched = sched
    return prm


def count(p, prm):
    v = lib().discover_count(p, C.byref(prm))
    if v < 0:
        _check(int(v))
    return int(v)


def decode(p, prm, cid):
    buf = C.create_string_buffer(4096)
    _check(lib().discover_decode(p, C.byref(prm), int(cid), buf, 4096))
    return buf.value.decode()


def decode_stats(t, cls):
    """Stats written to device memory (the byte tensor of a call with
    device_stats; cls = ScreenStats or L0Stats): a list of dicts, one per
    problem."""
    raw = bytes(t.cpu().numpy().tobytes())
    nb = len(raw) // C.sizeof(cls)
    arr = (cls * nb).from_buffer_copy(raw)
    return [arr[b].asdict() for b in range(nb)]


def _stream_handle(torch, device):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Context:
    """One library context on one HIP device."""

    def __init__(self, device=0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible: the discover library has no CPU path")
        self.torch = torch
        self.device = device
        self.h = C.c_void_p()
        _check(lib().discover_create(device, C.byref(self.h)))

    def close(self):
        if self.h:
            lib().discover_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ timing
    def set_timing(self, on=True):
        _check(lib().discover_set_timing(self.h, 1 if on else 0))

    def set_graph_timing(self, names=()):
        """Kernel timer names also timed inside captured graphs (replays)."""
        _check(lib().discover_set_graph_timing(self.h, ",".join(names).encode()))

    def reset_timing(self):
        _check(lib().discover_reset_timing(self.h))

    def set_fixup_capacity(self, entries):
        """Initial entries of the screening's exact fix-up lists."""
        _check(lib().discover_set_fixup_capacity(self.h, int(entries)))

    def set_rules(self, rules=None):
        """Selection rules of the following screening calls (None clears):
        {max_complexity: int (-1 none), forbid_nest: {op: [ops]} (the ops
        that may not be the top operator of op's operands), forbid_pairs:
        [[i, j], ...] (primary indices < 64 that may not appear together),
        target_units: [B] exponents over the problems' base units, or None}."""
        if rules is None:
            _check(lib().discover_set_rules(self.h, None))
            return
        r = Rules()
        r.max_complexity = int(rules.get("max_complexity", -1))
        for o, cs in (rules.get("forbid_nest") or {}).items():
            for c in cs:
                r.forbid_nest[OPS.index(o)] |= OP_BIT[c]
        pairs = [int(v) for pr in (rules.get("forbid_pairs") or ()) for v in pr]
        arr = (C.c_int32 * max(len(pairs), 1))(*pairs)
        r.n_forbid_pairs = len(pairs) // 2
        r.forbid_pairs = C.cast(arr, C.c_void_p) if pairs else None
        tu = rules.get("target_units")
        if tu is not None:
            if len(tu) > 8:
                raise ValueError("target_units: at most 8 base units")
            r.target_unit = 1
            for i, v in enumerate(tu):
                r.target_units[i] = int(v)
        _check(lib().discover_set_rules(self.h, C.byref(r)))

    def timing(self, kernel):
        n = C.c_int64()
        ms = C.c_double()
        _check(lib().discover_timing(self.h, kernel.encode(), C.byref(n), C.byref(ms)))
        return int(n.value), float(ms.value)

    # ------------------------------------------------------------ calls
    def _problems(self, Xs, Ys, units, excludes):
        """Problem structures of many datasets (and the objects they point to)."""
        import numpy as np
        nb = len(Xs)
        pbs = (Problem * nb)()
        keep = []
        for b in range(nb):
            pb = pbs[b]
            X = Xs[b].contiguous()
            Y = Ys[b].contiguous()
            keep += [X, Y]
            p_, n_ = X.shape
            pb.n, pb.p, pb.T = n_, p_, Y.shape[0]
            u = units[b] if units is not None else None
            if u is not None:
                u = np.ascontiguousarray(u, dtype=np.int32)
                keep.append(u)
                pb.B, pb.units = u.shape[1], u.ctypes.data
            else:
                pb.B = 0
            pb.X, pb.ldx = X.data_ptr(), n_
            pb.Y, pb.ldy = Y.data_ptr(), n_
            e = excludes[b] if excludes is not None else None
            if e is not None and e.numel():
                e = e.contiguous()
                keep.append(e)
                pb.exclude, pb.n_exclude = e.data_ptr(), e.numel()
        return pbs, keep

    def _stats(self, cls, nb, device_stats, dev):
        """Host stats structures, or a device byte tensor for them."""
        if device_stats:
            t = self.torch.zeros(nb * C.sizeof(cls), dtype=self.torch.uint8, device=dev)
            return t, t.data_ptr()
        st = (cls * nb)()
        return st, st

    def generate_screen(self, X, Y, prm, units=None, exclude=None, values=True, device_stats=False):
        """X [p][n], Y [T][n] float64 CUDA tensors; units [p][B] int32 host
        array or None; exclude int64 CUDA tensor of IDs or None.
        Returns (ids [T'][k], scores [T'][k], values [T'][k][n] or None, stats);
        with device_stats the call does not wait for the stream and stats is
        a device byte tensor (decode_stats)."""
        ((ids, sc, vals, st),) = self.generate_screen_batch(
            [X], [Y], prm, units=None if units is None else [units],
            excludes=None if exclude is None else [exclude], values=values, device_stats=device_stats)
        return ids, sc, vals, st

    def generate_screen_batch(self, Xs, Ys, prm, units=None, excludes=None, values=True,
                              device_stats=False):
        """One call over many datasets: Xs[b] [p_b][n_b], Ys[b] [T_b][n_b]
        float64 CUDA tensors; units[b] host [p_b][B] int32 or None;
        excludes[b] int64 CUDA tensor or None.  Returns per-dataset lists
        (ids [T'_b][k], scores, values [T'_b][k][n_max] or None, stats); with
        device_stats every stats entry is the call's device byte tensor."""
        torch = self.torch
        nb = len(Xs)
        dev = Xs[0].device
        tl = [1 if prm.score_mode == SCORE_MAX else y.shape[0] for y in Ys]
        rows = sum(tl)
        nmax = max(x.shape[1] for x in Xs)
        ids = torch.empty((rows, prm.k), dtype=torch.int64, device=dev)
        sc = torch.empty((rows, prm.k), dtype=torch.float64, device=dev)
        vals = torch.empty((rows, prm.k, nmax), dtype=torch.float64, device=dev) if values else None
        pbs, keep = self._problems(Xs, Ys, units, excludes)
        st, sp = self._stats(ScreenStats, nb, device_stats, dev)
        _check(lib().discover_generate_screen(
            self.h, pbs, nb, C.byref(prm), ids.data_ptr(), sc.data_ptr(),
            vals.data_ptr() if vals is not None else None, nmax, sp, _stream_handle(torch, dev)))
        out, r = [], 0
        for b in range(nb):
            out.append((ids[r:r + tl[b]], sc[r:r + tl[b]],
                        vals[r:r + tl[b], :, :Xs[b].shape[1]] if vals is not None else None,
                        st if device_stats else st[b].asdict()))
            r += tl[b]
        return out

    def reserve(self, Xs, Ys, prm, D_max=0, m=1, units=None, excludes=None):
        """Size the workspace for later asynchronous or captured calls of this
        screening shape, and L0 / OMP up to D_max dimensions (waits)."""
        pbs, keep = self._problems(Xs, Ys, units, excludes)
        _check(lib().discover_reserve(self.h, pbs, len(Xs), C.byref(prm), D_max, m,
                                      _stream_handle(self.torch, Xs[0].device)))

    def l0_fit_batch(self, Fs, idss, ys, D, m=1, resid=True, device_stats=False):
        """Exhaustive L0 of many subspaces in one call: Fs[b] [S_b][n_b],
        idss[b] [S_b] int64, ys[b] [n_b] (CUDA).  Returns per-dataset lists
        (subsets [m][D], rmse [m], coef [m][D+1], resid [m][n_b] or None, stats);
        with device_stats every stats entry is the call's device byte tensor."""
        torch = self.torch
        nb = len(Fs)
        Fs = [f.contiguous() for f in Fs]
        idss = [i.contiguous() for i in idss]
        ys = [y.contiguous() for y in ys]
        dev = Fs[0].device
        nmax = max(f.shape[1] for f in Fs)
        sub = torch.empty((nb, m, D), dtype=torch.int32, device=dev)
        rmse = torch.empty((nb, m), dtype=torch.float64, device=dev)
        coef = torch.empty((nb, m, D + 1), dtype=torch.float64, device=dev)
        res = torch.empty((nb, m, nmax), dtype=torch.float64, device=dev) if resid else None
        pbs = (L0Problem * nb)()
        for b in range(nb):
            S, n = Fs[b].shape
            pbs[b].n, pbs[b].S, pbs[b].F, pbs[b].ldf = n, S, Fs[b].data_ptr(), n
            pbs[b].ids, pbs[b].y = idss[b].data_ptr(), ys[b].data_ptr()
        st, sp = self._stats(L0Stats, nb, device_stats, dev)
        _check(lib().discover_l0_fit(self.h, pbs, nb, D, m, sub.data_ptr(), rmse.data_ptr(),
                                     coef.data_ptr(), res.data_ptr() if res is not None else None,
                                     nmax, sp, _stream_handle(torch, dev)))
        return [(sub[b], rmse[b], coef[b],
                 res[b, :, :Fs[b].shape[1]] if res is not None else None,
                 st if device_stats else st[b].asdict())
                for b in range(nb)]

    def l0_fit(self, F, ids, y, D, m=1, resid=True, device_stats=False):
        """F [S][n] float64, ids [S] int64, y [n] float64 (CUDA).  Returns
        (subsets [m][D] rows, rmse [m], coef [m][D+1], resid [m][n], stats)."""
        ((sub, rmse, coef, res, st),) = self.l0_fit_batch([F], [ids], [y], D, m, resid, device_stats)
        return sub, rmse, coef, res, st

    def l0_bnb_batch(self, Fs, idss, ys, D, m=1, resid=True, max_nodes=0):
        """Exact L0 by branch and bound (discover_l0_bnb) over many subspaces:
        Fs[b] [S_b][n_b], idss[b] [S_b] int64, ys[b] [n_b] (CUDA).  Returns per
        dataset (subsets [m][D] rows, rmse [m], coef [m][D+1], resid [m][n] or
        None, stats dict)."""
        torch = self.torch
        nb = len(Fs)
        Fs = [f.contiguous() for f in Fs]
        idss = [i.contiguous() for i in idss]
        ys = [y.contiguous() for y in ys]
        dev = Fs[0].device
        nmax = max(f.shape[1] for f in Fs)
        sub = torch.empty((nb, m, D), dtype=torch.int32, device=dev)
        rmse = torch.empty((nb, m), dtype=torch.float64, device=dev)
        coef = torch.empty((nb, m, D + 1), dtype=torch.float64, device=dev)
        res = torch.empty((nb, m, nmax), dtype=torch.float64, device=dev) if resid else None
        pbs = (L0Problem * nb)()
        for b in range(nb):
            S, n = Fs[b].shape
            pbs[b].n, pbs[b].S, pbs[b].F, pbs[b].ldf = n, S, Fs[b].data_ptr(), n
            pbs[b].ids, pbs[b].y = idss[b].data_ptr(), ys[b].data_ptr()
        st = (BnbStats * nb)()
        prm = BnbParams(int(max_nodes), 0)
        _check(lib().discover_l0_bnb(self.h, pbs, nb, D, m, C.byref(prm), sub.data_ptr(), rmse.data_ptr(),
                                     coef.data_ptr(), res.data_ptr() if res is not None else None, nmax, st,
                                     _stream_handle(torch, dev)))
        return [(sub[b], rmse[b], coef[b], res[b, :, :Fs[b].shape[1]] if res is not None else None,
                 st[b].asdict()) for b in range(nb)]

    def l0_bnb(self, F, ids, y, D, m=1, resid=True, max_nodes=0):
        """l0_bnb_batch for one subspace."""
        return self.l0_bnb_batch([F], [ids], [y], D, m, resid, max_nodes)[0]

    def anneal_batch(self, Fs, idss, ys, D, chains=4096, steps=10000, T0=0.01, alpha=0.9995, seed=0,
                     inits=None, chain_results=False, resid=False):
        """Simulated annealing over D-subsets of many subspaces in one call
        (discover_l0_anneal): Fs[b] [S_b][n_b], idss[b] [S_b] int64, ys[b]
        [n_b] (CUDA); inits: [nb][D] int32 rows or None.  Returns per dataset
        (rows [D] ascending, rmse, coef [D+1], energy, chain rows [chains][D]
        or None, chain energies [chains] or None, resid [n] or None)."""
        torch = self.torch
        nb = len(Fs)
        Fs = [f.contiguous() for f in Fs]
        idss = [i.contiguous() for i in idss]
        ys = [y.contiguous() for y in ys]
        dev = Fs[0].device
        nmax = max(f.shape[1] for f in Fs)
        rows = torch.empty((nb, D), dtype=torch.int32, device=dev)
        rmse = torch.empty(nb, dtype=torch.float64, device=dev)
        coef = torch.empty((nb, D + 1), dtype=torch.float64, device=dev)
        en = torch.empty(nb, dtype=torch.float64, device=dev)
        crow = torch.empty((nb, chains, D), dtype=torch.int32, device=dev) if chain_results else None
        cen = torch.empty((nb, chains), dtype=torch.float64, device=dev) if chain_results else None
        res = torch.empty((nb, nmax), dtype=torch.float64, device=dev) if resid else None
        pbs = (L0Problem * nb)()
        for b in range(nb):
            S, n = Fs[b].shape
            pbs[b].n, pbs[b].S, pbs[b].F, pbs[b].ldf = n, S, Fs[b].data_ptr(), n
            pbs[b].ids, pbs[b].y = idss[b].data_ptr(), ys[b].data_ptr()
        ini = None
        if inits is not None:
            ini = torch.as_tensor(inits, dtype=torch.int32, device=dev).reshape(nb, D).contiguous()
        prm = AnnealParams(chains, 0, steps, T0, alpha, seed & 0xFFFFFFFFFFFFFFFF)
        _check(lib().discover_l0_anneal(self.h, pbs, nb, D, C.byref(prm),
                                        ini.data_ptr() if ini is not None else None, rows.data_ptr(),
                                        rmse.data_ptr(), coef.data_ptr(), en.data_ptr(),
                                        crow.data_ptr() if crow is not None else None,
                                        cen.data_ptr() if cen is not None else None,
                                        res.data_ptr() if res is not None else None, nmax,
                                        _stream_handle(torch, dev)))
        return [(rows[b], rmse[b], coef[b], en[b], crow[b] if crow is not None else None,
                 cen[b] if cen is not None else None,
                 res[b, :Fs[b].shape[1]] if res is not None else None) for b in range(nb)]

    def anneal(self, F, ids, y, D, **kw):
        """anneal_batch for one subspace."""
        inits = kw.pop("init", None)
        return self.anneal_batch([F], [ids], [y], D, inits=None if inits is None else [inits], **kw)[0]

    def omp_noalloc(self, F, ids, y, D_max, init=None):
        """``omp`` through the allocation-free entry point (work space in the
        library's fixed per-GPU array; the outputs are allocated here)."""
        return self.omp(F, ids, y, D_max, init, _fn="discover_omp_noalloc")

    def omp(self, F, ids, y, D_max, init=None, _fn="discover_omp"):
        """OMP over the rows of F from the warm start ``init`` (int32 CUDA
        tensor of rows, or None).  Returns (active [D_max], coef [D_max+1],
        rmse, resid [n])."""
        torch = self.torch
        F = F.contiguous()
        S, n = F.shape
        dev = F.device
        act = torch.empty(D_max, dtype=torch.int32, device=dev)
        coef = torch.empty(D_max + 1, dtype=torch.float64, device=dev)
        rmse = torch.empty(1, dtype=torch.float64, device=dev)
        res = torch.empty(n, dtype=torch.float64, device=dev)
        pb = L0Problem()
        ids = ids.contiguous()
        y = y.contiguous()
        pb.n, pb.S, pb.F, pb.ldf, pb.ids, pb.y = n, S, F.data_ptr(), n, ids.data_ptr(), y.data_ptr()
        n_init = 0
        ip = None
        if init is not None and init.numel():
            init = init.to(torch.int32).contiguous()
            n_init = init.numel()
            ip = init.data_ptr()
        _check(getattr(lib(), _fn)(self.h, C.byref(pb), 1, D_max, ip, n_init, act.data_ptr(),
                                   coef.data_ptr(), rmse.data_ptr(), res.data_ptr(), n,
                                   _stream_handle(torch, dev)))
        return act, coef, rmse, res

    # ------------------------------------------------------------ loop
    def sisso_batch(self, Xs, ys, prm, D, n_resid=1):
        """The SISSO loop over many datasets at once: every dimension is one
        batched screening call and one batched L0 call.  Returns one result
        dict per dataset, shaped like ``sisso``'s."""
        torch = self.torch
        nb = len(Xs)
        dev = Xs[0].device
        S_ids = [torch.zeros(0, dtype=torch.int64, device=dev) for _ in range(nb)]
        F = [torch.zeros((0, x.shape[1]), dtype=torch.float64, device=dev) for x in Xs]
        targets = [y.reshape(1, -1) for y in ys]
        dims = [[] for _ in range(nb)]
        for d in range(1, D + 1):
            q = ScreenParams.from_buffer_copy(prm)
            if n_resid > 1 and d > 1:
                q.score_mode = SCORE_MAX
            scr = self.generate_screen_batch(Xs, targets, q, excludes=S_ids)
            for b in range(nb):
                ids, sc, vals, st = scr[b]
                ok = ids[0] >= 0
                S_ids[b] = torch.cat([S_ids[b], ids[0][ok]])
                F[b] = torch.cat([F[b], vals[0][ok]])
            fits = self.l0_fit_batch(F, S_ids, ys, d, n_resid)
            for b in range(nb):
                sub, rmse, coef, res, l0st = fits[b]
                ids, sc, vals, st = scr[b]
                dims[b].append({"sel_ids": ids[0], "sel_scores": sc[0], "screen_stats": st,
                                "subsets": sub, "rmse": rmse, "coef": coef, "l0_stats": l0st})
            targets = [fits[b][3] for b in range(nb)]
        return [{"dims": dims[b], "S_ids": S_ids[b], "F": F[b]} for b in range(nb)]

    def sisso_batch_graph(self, Xs, ys, prm, D, m=1, units=None, use_graph=True, omp_D=0):
        """The batched SISSO loop as one library call (discover_sisso_batch):
        the first call with given inputs runs eagerly and captures a
        hipGraph, later calls with the same input tensors replay it.  The
        output tensors are kept per input set and reused (and overwritten)
        by later calls.  Returns (ids [nb][D][k], scores [nb][D][k],
        subsets [nb][D][m][3], rmse [nb][D][m], coef [nb][D][m][4], replayed) with
        replayed 1 (graph replayed), 0 (eager) or -1 (eager; capture failed).
        With omp_D > D the best D-model of each dataset is extended by OMP
        and the result gains a seventh entry, (active [nb][omp_D] subspace
        rows, coef [nb][omp_D + 1], rmse [nb])."""
        torch = self.torch
        import numpy as np
        nb = len(Xs)
        dev = Xs[0].device
        key = (tuple(x.data_ptr() for x in Xs), tuple(y.data_ptr() for y in ys), D, m, prm.k, omp_D)
        cache = self.__dict__.setdefault("_sisso_out", {})
        if key not in cache:
            cache[key] = (torch.empty((nb, D, prm.k), dtype=torch.int64, device=dev),
                          torch.empty((nb, D, prm.k), dtype=torch.float64, device=dev),
                          torch.empty((nb, D, m, 3), dtype=torch.int32, device=dev),
                          torch.empty((nb, D, m), dtype=torch.float64, device=dev),
                          torch.empty((nb, D, m, 4), dtype=torch.float64, device=dev),
                          torch.empty((nb, max(omp_D, 1)), dtype=torch.int32, device=dev),
                          torch.empty((nb, max(omp_D, 1) + 1), dtype=torch.float64, device=dev),
                          torch.empty((nb,), dtype=torch.float64, device=dev))
        ids, sc, sub, rmse, coef, oact, ocoef, ormse = cache[key]
        pbs = (Problem * nb)()
        keep = []
        for b in range(nb):
            x, y = Xs[b], ys[b]
            assert x.is_contiguous() and y.is_contiguous()
            p_, n_ = x.shape
            pbs[b].n, pbs[b].p, pbs[b].T = n_, p_, 1
            u = units[b] if units is not None else None
            if u is not None:
                u = np.ascontiguousarray(u, dtype=np.int32)
                keep.append(u)
                pbs[b].B, pbs[b].units = u.shape[1], u.ctypes.data
            pbs[b].X, pbs[b].ldx = x.data_ptr(), n_
            pbs[b].Y, pbs[b].ldy = y.data_ptr(), n_
        rep = C.c_int32(0)
        po = (oact.data_ptr(), ocoef.data_ptr(), ormse.data_ptr()) if omp_D else (None, None, None)
        _check(lib().discover_sisso_batch(self.h, pbs, nb, C.byref(prm), D, m, 1 if use_graph else 0,
                                          ids.data_ptr(), sc.data_ptr(), sub.data_ptr(),
                                          rmse.data_ptr(), coef.data_ptr(), omp_D, po[0], po[1], po[2],
                                          C.byref(rep), _stream_handle(torch, dev)))
        if rep.value < 0:
            self.capture_error = lib().discover_last_error().decode()
        if omp_D:
            return ids, sc, sub, rmse, coef, int(rep.value), (oact, ocoef, ormse)
        return ids, sc, sub, rmse, coef, int(rep.value)

    def sisso(self, X, y, prm, D, units=None, n_resid=1, omp_D=0):
        """The SISSO loop: for d = 1..D screen against the residual(s) of the
        best dimension-(d-1) model(s) (the target at d = 1), append the k
        selected features to the subspace, and fit the original y by
        exhaustive L0 over all d-subsets.  Optionally extend the D-model by
        OMP to omp_D features.  X [p][n], y [n] CUDA float64."""
        torch = self.torch
        dev = X.device
        S_ids = torch.zeros(0, dtype=torch.int64, device=dev)
        F = torch.zeros((0, X.shape[1]), dtype=torch.float64, device=dev)
        targets = y.reshape(1, -1)
        dims = []
        for d in range(1, D + 1):
            q = ScreenParams.from_buffer_copy(prm)
            if targets.shape[0] > 1:
                q.score_mode = SCORE_MAX
            ids, sc, vals, st = self.generate_screen(X, targets, q, units=units, exclude=S_ids)
            ok = ids[0] >= 0
            S_ids = torch.cat([S_ids, ids[0][ok]])
            F = torch.cat([F, vals[0][ok]])
            m = n_resid
            sub, rmse, coef, res, l0st = self.l0_fit(F, S_ids, y, d, m)
            dims.append({"sel_ids": ids[0], "sel_scores": sc[0], "screen_stats": st,
                         "subsets": sub, "rmse": rmse, "coef": coef, "l0_stats": l0st})
            targets = res
        out = {"dims": dims, "S_ids": S_ids, "F": F}
        if omp_D > D:
            act, coef, rmse, res = self.omp(F, S_ids, y, omp_D, dims[-1]["subsets"][0])
            out["omp"] = {"active": act, "coef": coef, "rmse": rmse, "resid": res}
        return out
