"""Python binding of librtdetmcd: argument marshalling only.

Tensors live on the GPU; every step runs in the library's HIP kernels on the
current torch stream.  The library must be built (``python -m
paper_1910_05615_amd.build``); nothing here falls back to a CPU path.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
from typing import List, Optional, Sequence

import torch

from . import _lib

_handles = {}

STD = {"unimcd": 0, "medmad": 1}
CSTEP = {"full": 0, "update": 1, "auto": 2, "smw": 3}
DIST = {"cholesky": 0, "inverse": 1}
START_WARM = 2   # block_start of a block fitted from a warm start (RTDETMCD_START_WARM)
POOL = {"printed": 0, "union": 1}
LAUNCH = {"batched": 0, "plain": 1}


class RTDetMCDError(RuntimeError):
    pass


def _handle(device: torch.device):
    lib = _lib.load()
    idx = device.index if device.index is not None else torch.cuda.current_device()
    h = _handles.get(idx)
    if h is None:
        hv = C.c_void_p()
        st = lib.rtdetmcd_create(C.byref(hv), idx, None)
        if st != 0:
            raise RTDetMCDError(f"rtdetmcd_create failed ({_lib.STATUS_NAMES.get(st, st)})")
        h = hv.value
        _handles[idx] = h
    stream = torch.cuda.current_stream(device).cuda_stream
    lib.rtdetmcd_set_stream(h, C.c_void_p(stream))
    return lib, h


def _check(lib, h, st, what):
    if st != 0:
        msg = lib.rtdetmcd_last_error(h)
        raise RTDetMCDError(f"{what}: {_lib.STATUS_NAMES.get(st, st)}: "
                            f"{msg.decode() if msg else ''}")


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dtype_code(X: torch.Tensor) -> int:
    if X.dtype == torch.float32:
        return 0
    if X.dtype == torch.float64:
        return 1
    raise TypeError("X must be float32 or float64")


def _check_X(X: torch.Tensor):
    if not X.is_cuda:
        raise ValueError("X must be a CUDA (HIP) tensor")
    if X.dim() != 2 or (X.numel() > 0 and X.stride(1) != 1):   # empty: any strides
        raise ValueError("X must be 2-D with unit column stride")


def make_opts(alpha: float = 0.75, standardize: str = "unimcd", cstep_mode: str = "auto",
              max_csteps: int = 100, kappa_max: float = 1000.0, cutoff_q: float = 0.975,
              pool: str = "printed", rew_consistency: bool = False, omega: int = 4096,
              launch: str = "batched", graph: bool = False, rounds_per_sync: int = 4,
              distance: str = "cholesky", tune: bool = False) -> _lib.Opts:
    lib = _lib.load()
    o = _lib.Opts()
    lib.rtdetmcd_default_opts(C.byref(o))
    o.alpha = alpha
    o.standardize = STD[standardize]
    o.cstep_mode = CSTEP[cstep_mode]
    o.max_csteps = max_csteps
    o.kappa_max = kappa_max
    o.cutoff_q = cutoff_q
    o.pool_mode = POOL[pool]
    o.rew_consistency = int(rew_consistency)
    o.omega = omega
    o.launch = LAUNCH[launch]
    o.graph = int(graph)
    o.rounds_per_sync = rounds_per_sync
    o.distance = DIST[distance]
    o.tune = int(tune)
    return o


def plan(n: int, p: int, h_sub: int = 0, n_chunks: int = 0, **opts):
    return _plan_o(_lib.load(), n, p, h_sub, n_chunks, make_opts(**opts))


def _plan_o(lib, n: int, p: int, h_sub: int, n_chunks: int, o):
    q, m, h = C.c_int32(), C.c_int64(), C.c_int64()
    st = lib.rtdetmcd_plan(n, p, h_sub, n_chunks, C.byref(o), C.byref(q), C.byref(m), C.byref(h))
    if st != 0:
        raise RTDetMCDError(f"rtdetmcd_plan: {_lib.STATUS_NAMES.get(st, st)}")
    return q.value, m.value, h.value


def chi2_quantile(q: float, df: int) -> float:
    return _lib.load().rtdetmcd_chi2_quantile(q, df)


def chi2_cdf(x: float, df: int) -> float:
    return _lib.load().rtdetmcd_chi2_cdf(x, df)


def consistency(alpha: float, p: int) -> float:
    return _lib.load().rtdetmcd_consistency(alpha, p)


# ----------------------------------------------------------------- low-level steps

def distances(X: torch.Tensor, mu: torch.Tensor, L: torch.Tensor) -> torch.Tensor:
    """Squared distances ||L^{-1}(x_i - mu)||^2 of the rows of X (float64 output)."""
    _check_X(X)
    n, p = X.shape
    lib, h = _handle(X.device)
    mu = mu.to(device=X.device, dtype=torch.float64).contiguous()
    L = L.to(device=X.device, dtype=torch.float64).contiguous()
    d2 = torch.empty(n, dtype=torch.float64, device=X.device)
    st = lib.rtdetmcd_distances(h, _ptr(X), _dtype_code(X), n, p, X.stride(0), _ptr(mu),
                                _ptr(L), _ptr(d2))
    _check(lib, h, st, "rtdetmcd_distances")
    return d2


def distances_into(X: torch.Tensor, mu: torch.Tensor, L: torch.Tensor, d2: torch.Tensor) -> None:
    """distances() into a preallocated float64 output; mu and L float64,
    contiguous, on X's device (no allocation; for timing loops)."""
    n, p = X.shape
    lib, h = _handle(X.device)
    st = lib.rtdetmcd_distances(h, _ptr(X), _dtype_code(X), n, p, X.stride(0), _ptr(mu),
                                _ptr(L), _ptr(d2))
    _check(lib, h, st, "rtdetmcd_distances")


def select(d2: torch.Tensor, h_sub: int):
    """(ascending indices of the h_sub smallest d2, 0/1 mask); ties by index."""
    d2 = d2.to(torch.float64).contiguous()
    m = d2.numel()
    lib, h = _handle(d2.device)
    idx = torch.empty(h_sub, dtype=torch.int32, device=d2.device)
    mask = torch.empty(m, dtype=torch.uint8, device=d2.device)
    st = lib.rtdetmcd_select(h, _ptr(d2), m, h_sub, _ptr(idx), _ptr(mask))
    _check(lib, h, st, "rtdetmcd_select")
    return idx, mask


@dataclasses.dataclass
class CStepResult:
    mu: torch.Tensor
    sigma: torch.Tensor
    hsubset: torch.Tensor
    status: int
    iters: int
    logdet: float


def cstep(X: torch.Tensor, h_sub: int, mu0: torch.Tensor, sigma0: torch.Tensor,
          kappa_scale: Optional[torch.Tensor] = None, noalloc: bool = False,
          **opts) -> CStepResult:
    """C-steps on one block from (mu0, sigma0) until the h-subset repeats.
    noalloc: run rtdetmcd_cstep_noalloc (no device allocation in the library;
    m <= 131072)."""
    _check_X(X)
    m, p = X.shape
    lib, h = _handle(X.device)
    o = make_opts(**opts)
    dev = X.device
    mu0 = mu0.to(device=dev, dtype=torch.float64).contiguous()
    sigma0 = sigma0.to(device=dev, dtype=torch.float64).contiguous()
    ks = None if kappa_scale is None else kappa_scale.to(device=dev, dtype=torch.float64).contiguous()
    mu = torch.empty(p, dtype=torch.float64, device=dev)
    sig = torch.empty(p, p, dtype=torch.float64, device=dev)
    hs = torch.empty(h_sub, dtype=torch.int32, device=dev)
    stt = torch.empty(1, dtype=torch.int32, device=dev)
    its = torch.empty(1, dtype=torch.int32, device=dev)
    ld = torch.empty(1, dtype=torch.float64, device=dev)
    fn = lib.rtdetmcd_cstep_noalloc if noalloc else lib.rtdetmcd_cstep
    st = fn(h, _ptr(X), _dtype_code(X), m, p, X.stride(0), h_sub, _ptr(mu0), _ptr(sigma0),
            _ptr(ks), C.byref(o), _ptr(mu), _ptr(sig), _ptr(hs), _ptr(stt), _ptr(its), _ptr(ld))
    _check(lib, h, st, "rtdetmcd_cstep_noalloc" if noalloc else "rtdetmcd_cstep")
    return CStepResult(mu, sig, hs, int(stt.item()), int(its.item()), float(ld.item()))


PROF_KINDS = {"segsort": 0, "cstep_dist": 1, "select": 2, "sscp": 3, "finalize": 4,
              "final_dist": 5, "fit": 6, "distances": 7}


def profile(enable: bool, device=None) -> None:
    """Start (clearing earlier records) or stop the library's kernel timing
    on this device's handle (rtdetmcd_profile)."""
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    lib, h = _handle(dev)
    _check(lib, h, lib.rtdetmcd_profile(h, int(bool(enable))), "rtdetmcd_profile")


def profile_read(device=None) -> dict:
    """Totals per kernel class since profile(True): {name: {ms, launches,
    bytes, flops_useful, flops_exec}} (rtdetmcd_profile_read)."""
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    lib, h = _handle(dev)
    out = {}
    for name, k in PROF_KINDS.items():
        ms, n, b, fu, fe = C.c_double(), C.c_int64(), C.c_double(), C.c_double(), C.c_double()
        _check(lib, h, lib.rtdetmcd_profile_read(h, k, C.byref(ms), C.byref(n), C.byref(b),
                                                 C.byref(fu), C.byref(fe)),
               "rtdetmcd_profile_read")
        out[name] = {"ms": ms.value, "launches": n.value, "bytes": b.value,
                     "flops_useful": fu.value, "flops_exec": fe.value}
    return out


def tuned_plans(device=None) -> list:
    """The autotuned C-step plans of this device's handle (opts tune=True),
    most recent last: [(p bucket, rows per distance tile, items per distance
    tile, C-steps of the last fit)] (rtdetmcd_tuned_plans)."""
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    lib, h = _handle(dev)
    cnt = C.c_int32()
    _check(lib, h, lib.rtdetmcd_tuned_plans(h, None, 0, C.byref(cnt)), "rtdetmcd_tuned_plans")
    buf = (C.c_int64 * (4 * max(1, cnt.value)))()
    _check(lib, h, lib.rtdetmcd_tuned_plans(h, buf, cnt.value, C.byref(cnt)),
           "rtdetmcd_tuned_plans")
    return [tuple(int(buf[4 * k + j]) for j in range(4)) for k in range(cnt.value)]


def sort_reruns(device=None) -> int:
    """Fits on this device's handle that were run again with ballot ranking
    after a sort's order check failed (rtdetmcd_sort_reruns)."""
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    lib, h = _handle(dev)
    return int(lib.rtdetmcd_sort_reruns(h))


# ----------------------------------------------------------------- full fit

@dataclasses.dataclass
class Fit:
    mu: torch.Tensor
    sigma: torch.Tensor
    mu_raw: torch.Tensor
    sigma_raw: torch.Tensor
    logdet: torch.Tensor          # [log det sigma_raw, log det sigma]
    dist: torch.Tensor
    outlier: torch.Tensor
    hsubset: torch.Tensor         # q x h
    block_status: torch.Tensor
    block_start: torch.Tensor
    block_iters: torch.Tensor
    loc: torch.Tensor
    scale: torch.Tensor
    n_w: torch.Tensor
    rew_mask: torch.Tensor        # rows kept by the reweighting (u8)
    q: int
    m: int
    h: int
    c_rew: float = 1.0            # factor of the reweighted scatter
    # diagnostics (fit(..., diagnostics=True)): log det of each block's chosen
    # start at each evaluated C-step (q x max_csteps, NaN beyond block_iters),
    # the gap d2_(h+1) - d2_(h) of its last distances (q), and the smallest
    # |dist^2 - chi2| of the final distances (1)
    ldtrace: Optional[torch.Tensor] = None
    hmargin: Optional[torch.Tensor] = None
    cmargin: Optional[torch.Tensor] = None


def _alloc_fit(X: torch.Tensor, q: int, m: int, h: int):
    """The outputs of one fit: one device allocation per element type, the
    outputs slices of it (four allocator calls per fit instead of fifteen)."""
    n, p = X.shape
    dev = X.device
    pp = p * p
    f = torch.empty(4 * p + 2 * pp + 2 + n, dtype=torch.float64, device=dev)
    i = torch.empty(q * h + 3 * q, dtype=torch.int32, device=dev)
    u = torch.empty(2 * n, dtype=torch.uint8, device=dev)
    F = Fit(mu=f[0:p], sigma=f[p:p + pp].view(p, p), mu_raw=f[p + pp:2 * p + pp],
            sigma_raw=f[2 * p + pp:2 * p + 2 * pp].view(p, p),
            logdet=f[2 * p + 2 * pp:2 * p + 2 * pp + 2],
            loc=f[2 * p + 2 * pp + 2:3 * p + 2 * pp + 2],
            scale=f[3 * p + 2 * pp + 2:4 * p + 2 * pp + 2], dist=f[4 * p + 2 * pp + 2:],
            hsubset=i[:q * h].view(q, h), block_status=i[q * h:q * h + q],
            block_start=i[q * h + q:q * h + 2 * q], block_iters=i[q * h + 2 * q:],
            outlier=u[:n], rew_mask=u[n:], n_w=torch.empty(1, dtype=torch.int64, device=dev),
            q=q, m=m, h=h)
    out = _lib.Out(mu=F.mu.data_ptr(), sigma=F.sigma.data_ptr(), mu_raw=F.mu_raw.data_ptr(),
                   sigma_raw=F.sigma_raw.data_ptr(), logdet=F.logdet.data_ptr(),
                   dist=F.dist.data_ptr(), outlier=F.outlier.data_ptr(),
                   hsubset=F.hsubset.data_ptr(), block_status=F.block_status.data_ptr(),
                   block_start=F.block_start.data_ptr(), block_iters=F.block_iters.data_ptr(),
                   loc=F.loc.data_ptr(), scale=F.scale.data_ptr(), n_w=F.n_w.data_ptr(),
                   rew_mask=F.rew_mask.data_ptr())
    return F, out


def _alloc_diag(fits, outs, maxs: int):
    """The diagnostics outputs of fits (one float64 allocation for all)."""
    sz = [F.q * maxs + F.q + 1 for F in fits]
    d_all = torch.empty(sum(sz), dtype=torch.float64, device=fits[0].mu.device)
    base = d_all.data_ptr()
    off = 0
    for F, out, part in zip(fits, outs, d_all.split(sz)):
        q = F.q
        tr, hm, cm = part.split([q * maxs, q, 1])
        F.ldtrace, F.hmargin, F.cmargin = tr.view(q, maxs), hm, cm
        out.ldtrace = base + 8 * off
        out.hmargin = base + 8 * (off + q * maxs)
        out.cmargin = base + 8 * (off + q * maxs + q)
        off += q * maxs + q + 1


def _alloc_fits(Xs, plans):
    """The outputs of many fits: one device allocation per element type for
    the whole batch, cut into every fit's outputs by one split per type (the
    views are the Fit tensors); the pointers handed to the library are
    computed from the offsets."""
    dev = Xs[0].device
    fsz, isz, usz = [], [], []
    for X, (q, m, h) in zip(Xs, plans):
        n, p = X.shape
        pp = p * p
        fsz += [p, pp, p, pp, 2, p, p, n]
        isz += [q * h, q, q, q]
        usz += [n, n]
    k = len(Xs)
    f_all = torch.empty(sum(fsz), dtype=torch.float64, device=dev)
    i_all = torch.empty(sum(isz), dtype=torch.int32, device=dev)
    u_all = torch.empty(sum(usz), dtype=torch.uint8, device=dev)
    w_all = torch.empty(k, dtype=torch.int64, device=dev)
    fb, ib, ub, wb = f_all.data_ptr(), i_all.data_ptr(), u_all.data_ptr(), w_all.data_ptr()
    fv, iv, uv, wv = f_all.split(fsz), i_all.split(isz), u_all.split(usz), w_all.split(1)
    fits, outs = [], []
    fo = io = uo = 0
    for j, (X, (q, m, h)) in enumerate(zip(Xs, plans)):
        n, p = X.shape
        pp = p * p
        mu, sg, mr, sr, ld, loc, sc, dist = fv[8 * j:8 * j + 8]
        hs, bst, bsa, bit = iv[4 * j:4 * j + 4]
        F = Fit(mu=mu, sigma=sg.view(p, p), mu_raw=mr, sigma_raw=sr.view(p, p), logdet=ld,
                loc=loc, scale=sc, dist=dist, hsubset=hs.view(q, h), block_status=bst,
                block_start=bsa, block_iters=bit, outlier=uv[2 * j], rew_mask=uv[2 * j + 1],
                n_w=wv[j], q=q, m=m, h=h)
        f0, i0, u0 = fb + 8 * fo, ib + 4 * io, ub + uo
        outs.append(_lib.Out(mu=f0, sigma=f0 + 8 * p, mu_raw=f0 + 8 * (p + pp),
                             sigma_raw=f0 + 8 * (2 * p + pp), logdet=f0 + 8 * (2 * p + 2 * pp),
                             loc=f0 + 8 * (2 * p + 2 * pp + 2),
                             scale=f0 + 8 * (3 * p + 2 * pp + 2),
                             dist=f0 + 8 * (4 * p + 2 * pp + 2), hsubset=i0,
                             block_status=i0 + 4 * q * h, block_start=i0 + 4 * (q * h + q),
                             block_iters=i0 + 4 * (q * h + 2 * q), outlier=u0, rew_mask=u0 + n,
                             n_w=wb + 8 * j))
        fits.append(F)
        fo += 4 * p + 2 * pp + 2 + n
        io += q * h + 3 * q
        uo += 2 * n
    return fits, outs


def random_partition(n: int, seed: int, device=None) -> torch.Tensor:
    """A random permutation of the n rows (int32, on `device`) for the random
    partition of Sec. 4: block l of a fit given ``perm`` is rows
    perm[l m : (l+1) m].  Drawn on the host from a seeded torch generator, so
    that the same rows can be handed to any other implementation."""
    g = torch.Generator().manual_seed(int(seed))
    return torch.randperm(n, generator=g, dtype=torch.int64).to(torch.int32).to(device)


def fit(X: torch.Tensor, h_sub: int = 0, n_chunks: int = 0,
        perm: Optional[torch.Tensor] = None, warm=None, diagnostics: bool = False,
        **opts) -> Fit:
    """RT-DetMCD fit of X (n x p) on the GPU; all outputs stay on the device.

    perm: optional int32 device tensor of n row indices, the random partition
    of Sec. 4 (see random_partition); None gives contiguous blocks.
    warm: optional (mu, sigma) of a previous fit (units of X), the warm start
    of the last paragraph of Sec. 4.
    diagnostics: also return the log det trace, selection gaps and flag
    margin (Fit.ldtrace, hmargin, cmargin)."""
    if perm is not None or warm is not None:
        fits, status = fit_batched([X], h_subs=[h_sub], n_chunks=[n_chunks], perms=[perm],
                                   warms=[warm], diagnostics=diagnostics, **opts)
        if status[0] != 0:
            lib, hd = _handle(X.device)
            _check(lib, hd, status[0], "rtdetmcd_fit_batched")
        return fits[0]
    _check_X(X)
    n, p = X.shape
    q, m, h = plan(n, p, h_sub, n_chunks, **opts)
    lib, hd = _handle(X.device)
    o = make_opts(**opts)
    F, out = _alloc_fit(X, q, m, h)
    if diagnostics:
        _alloc_diag([F], [out], o.max_csteps)
    F.c_rew = lib.rtdetmcd_consistency(o.cutoff_q, p) if o.rew_consistency else 1.0
    st = lib.rtdetmcd_fit(hd, _ptr(X), _dtype_code(X), n, p, X.stride(0), h_sub, n_chunks,
                          C.byref(o), C.byref(out))
    _check(lib, hd, st, "rtdetmcd_fit")
    return F


def backward(X: torch.Tensor, F: Fit, g_dist: Optional[torch.Tensor] = None,
             g_mu: Optional[torch.Tensor] = None,
             g_sigma: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Gradient with respect to X (float64, n x p) of <g_dist, dist> +
    <g_mu, mu> + <g_sigma, sigma> for the fit F of X, with the h-subsets and
    the reweighting set held fixed (rtdetmcd_backward)."""
    _check_X(X)
    n, p = X.shape
    lib, hd = _handle(X.device)

    def cot(t, shape):
        if t is None:
            return None
        t = t.to(device=X.device, dtype=torch.float64).contiguous()
        if tuple(t.shape) != shape:
            raise ValueError(f"cotangent of shape {tuple(t.shape)}, expected {shape}")
        return t

    gd, gm, gs = cot(g_dist, (n,)), cot(g_mu, (p,)), cot(g_sigma, (p, p))
    gX = torch.empty(n, p, dtype=torch.float64, device=X.device)
    st = lib.rtdetmcd_backward(hd, _ptr(X), _dtype_code(X), n, p, X.stride(0), _ptr(F.mu),
                               _ptr(F.sigma), _ptr(F.dist), _ptr(F.rew_mask), _ptr(F.n_w),
                               float(F.c_rew), _ptr(gd), _ptr(gm), _ptr(gs), _ptr(gX))
    _check(lib, hd, st, "rtdetmcd_backward")
    return gX


class RobustMCD(torch.autograd.Function):
    """(mu, sigma, dist) of an RT-DetMCD fit as a differentiable function of X.

    The backward holds the h-subsets and the reweighting set fixed; the fit is
    piecewise smooth in X and this is its derivative wherever it exists.
    ``fit_kw`` is a dict of keyword arguments of ``fit``."""

    @staticmethod
    def forward(ctx, X, fit_kw=None):
        F = fit(X.detach(), **(fit_kw or {}))
        ctx.save_for_backward(X)
        ctx.fit_result = F
        return F.mu, F.sigma, F.dist

    @staticmethod
    def backward(ctx, g_mu, g_sigma, g_dist):
        (X,) = ctx.saved_tensors
        gX = backward(X.detach(), ctx.fit_result, g_dist, g_mu, g_sigma)
        return gX.to(X.dtype), None


def fit_batched(Xs: Sequence[torch.Tensor], h_subs: Optional[Sequence[int]] = None,
                n_chunks: Optional[Sequence[int]] = None,
                perms: Optional[Sequence[Optional[torch.Tensor]]] = None,
                warms: Optional[Sequence] = None, diagnostics: bool = False, **opts):
    """Fit many independent datasets in the same launches.

    perms: optional per-dataset random partitions (int32 device tensors of n
    row indices, or None).  warms: optional per-dataset warm starts ((mu,
    sigma) in the units of X, or None).  diagnostics: as in fit.  Returns
    (list of Fit, list of per-dataset status codes)."""
    lib, hd = _handle(Xs[0].device)
    o = make_opts(**opts)
    k = len(Xs)
    h_subs = list(h_subs) if h_subs is not None else [0] * k
    n_chunks = list(n_chunks) if n_chunks is not None else [0] * k
    perms = list(perms) if perms is not None else [None] * k
    warms = list(warms) if warms is not None else [None] * k
    arr = (_lib.DatasetDesc * k)()
    keep = []   # warm-start tensors stay alive until the call returns
    plans = []
    for i, X in enumerate(Xs):
        _check_X(X)
        n, p = X.shape
        plans.append(_plan_o(lib, n, p, h_subs[i], n_chunks[i], o))
    fits, outs = _alloc_fits(Xs, plans) if k else ([], [])
    if diagnostics and k:
        _alloc_diag(fits, outs, o.max_csteps)
    for i, X in enumerate(Xs):
        n, p = X.shape
        F, out = fits[i], outs[i]
        F.c_rew = lib.rtdetmcd_consistency(o.cutoff_q, p) if o.rew_consistency else 1.0
        pm = perms[i]
        if pm is not None:
            if (pm.dtype != torch.int32 or pm.device != X.device or pm.dim() != 1
                    or pm.shape[0] != n or not pm.is_contiguous()):
                raise ValueError("perm must be a contiguous int32 tensor of n rows on X's device")
        wm = ws = None
        if warms[i] is not None:
            wm = warms[i][0].to(device=X.device, dtype=torch.float64).contiguous()
            ws = warms[i][1].to(device=X.device, dtype=torch.float64).contiguous()
            if tuple(wm.shape) != (p,) or tuple(ws.shape) != (p, p):
                raise ValueError("warm start must be (mu [p], sigma [p, p])")
            keep += [wm, ws]
        arr[i] = _lib.DatasetDesc(X=X.data_ptr(), dtype=_dtype_code(X), n=n, p=p, ld=X.stride(0),
                                  h_sub=h_subs[i], n_chunks=n_chunks[i], out=out,
                                  perm=pm.data_ptr() if pm is not None else None,
                                  warm_mu=wm.data_ptr() if wm is not None else None,
                                  warm_sigma=ws.data_ptr() if ws is not None else None)
    status = (C.c_int32 * k)()
    st = lib.rtdetmcd_fit_batched(hd, k, arr, C.byref(o), status)
    _check(lib, hd, st, "rtdetmcd_fit_batched")
    return fits, [int(s) for s in status]


def score(X: torch.Tensor, mu: torch.Tensor, Linv: torch.Tensor, cut: float = 0.0):
    """Distances and flags of the rows of X against a stored fit (mu, Linv).

    Linv is the inverse lower Cholesky factor of Sigma; cut <= 0 uses
    chi2_{p,0.975}.  Returns (dist float64 [n], outlier uint8 [n])."""
    _check_X(X)
    n, p = X.shape
    lib, h = _handle(X.device)
    mu = mu.to(device=X.device, dtype=torch.float64).contiguous()
    Linv = Linv.to(device=X.device, dtype=torch.float64).contiguous()
    dist = torch.empty(n, dtype=torch.float64, device=X.device)
    flag = torch.empty(n, dtype=torch.uint8, device=X.device)
    st = lib.rtdetmcd_score(h, _ptr(X), _dtype_code(X), n, p, X.stride(0), _ptr(mu), _ptr(Linv),
                            float(cut), _ptr(dist), _ptr(flag))
    _check(lib, h, st, "rtdetmcd_score")
    return dist, flag


def score_into(X: torch.Tensor, mu: torch.Tensor, Linv: torch.Tensor, dist: torch.Tensor,
               flag: torch.Tensor, cut: float = 0.0) -> None:
    """score() into preallocated outputs (no allocation; for timing loops)."""
    n, p = X.shape
    lib, h = _handle(X.device)
    st = lib.rtdetmcd_score(h, _ptr(X), _dtype_code(X), n, p, X.stride(0), _ptr(mu), _ptr(Linv),
                            float(cut), _ptr(dist), _ptr(flag))
    _check(lib, h, st, "rtdetmcd_score")
