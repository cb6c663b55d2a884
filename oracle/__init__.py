"""CPU oracle for the LLR energy-restricted sweep (test infrastructure only).

This package wraps ``llr_oracle.c``, a plain FP64 C implementation of the
method of arXiv:1509.08391 (Sec. 2.2 restricted expectation values and the
Robbins-Monro iteration, Algorithm 1, Sec. 2.5 replica exchange, Sec. 3.1
compact U(1) model, eqs. (kk3a), (l19)-(l20) reconstruction).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import it.  It shares no code with the GPU library.

Conventions (identical on both sides, written independently):
  * canonical link layout: ``theta[chain, mu, s]``, s = x0 + L x1 + L^2 x2 + ...
  * colour c = 2 mu + p (p = site parity), heatbath colours 0..2d-1 then
    overrelaxation colours 0..2d-1 per sweep
  * Philox4x32-10 key = (seed lo, seed hi); counter = (h or link index,
    attempt|colour<<8|kind<<12|lattice<<16, sweep, interval)
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "llr_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

KIND_SWEEP, KIND_INIT, KIND_APPROACH, KIND_REPLICA, KIND_MLP, KIND_BOOT, KIND_MUCA = 0, 1, 2, 3, 4, 5, 6
MODE_RESTRICTED, MODE_APPROACH, MODE_FREE, MODE_MUCA, MODE_LINK = 0, 1, 2, 3, 4
# order of the class passes in a sweep: heatbath of every colour then
# overrelaxation of every colour, or heatbath and overrelaxation per colour,
# or the grouped order on the first ceil(n/2) chains of a lattice and
# overrelaxation of every colour then heatbath of every colour on the others
SWEEP_GROUPED, SWEEP_INTERLEAVED, SWEEP_STAGGERED = 0, 1, 2
N_PARAMS = 4417


_GCC = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-fno-fast-math"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        subprocess.check_call(_GCC + [_SRC, "-o", _LIB_PATH + ".tmp", "-lm"])
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def build_variant(path: str, defines) -> "C.CDLL":
    """A copy of the oracle compiled with extra preprocessor macros (the pins'
    planted mistakes, e.g. OR_PLANT_RE_SIGN) at `path`; wrappers take it as
    their `use` argument."""
    subprocess.check_call(_GCC + [f"-D{m}" for m in defines] + [_SRC, "-o", path, "-lm"])
    v = C.CDLL(path)
    _declare(v)
    return v


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = C.CDLL(_LIB_PATH)
        _declare(_lib)
    return _lib


def _p(t):
    return C.POINTER(t)


class RunParams(C.Structure):
    _fields_ = [("d", C.c_int), ("L", C.c_int), ("n", C.c_int),
                ("n_th", C.c_int), ("n_a", C.c_int), ("n_rm", C.c_int),
                ("recompute_every", C.c_int), ("approach_cap", C.c_int),
                ("replica_exchange", C.c_int), ("f32", C.c_int), ("lattice_id", C.c_int),
                ("hot_start", C.c_int), ("seed", C.c_uint64),
                ("dE", C.c_double), ("w", C.c_double), ("eps", C.c_double), ("link", C.c_int),
                ("interleave", C.c_int)]


class RunOut(C.Structure):
    _fields_ = [("a", _p(C.c_double)), ("a_hist", _p(C.c_double)), ("theta", _p(C.c_double)),
                ("E", _p(C.c_double)), ("conf", _p(C.c_int)), ("conv_iter", _p(C.c_int)),
                ("conv_sweeps", _p(C.c_longlong)), ("approach_sweeps", _p(C.c_longlong)),
                ("bits", _p(C.c_uint16)), ("sumE_hist", _p(C.c_double)),
                ("re_acc", _p(C.c_longlong))]


def _declare(L):
    d, i, u32, u64, l = C.c_double, C.c_int, C.c_uint32, C.c_uint64, C.c_long
    L.or_philox_batch.argtypes = [l, _p(u32), _p(u32), _p(u32)]
    L.or_uniforms.argtypes = [l, _p(u32), i, _p(d), _p(d)]
    L.or_neighbour.argtypes = [i, i, l, i, i]
    L.or_neighbour.restype = l
    L.or_energy.argtypes = [i, i, _p(d)]
    L.or_energy.restype = d
    L.or_adjoint.argtypes = [i, i, _p(d)]
    L.or_adjoint.restype = d
    L.or_local_field.argtypes = [i, i, _p(d), i, l, _p(d), _p(d)]
    L.or_vonmises_batch.argtypes = [l, d, u64, u32, u32, u32, i, _p(d), _p(i), _p(d)]
    L.or_hot_start.argtypes = [i, i, i, u64, i, i, _p(d)]
    L.or_link_draw_batch.argtypes = [l, d, d, d, u64, u32, u32, i, _p(d), _p(i)]
    L.or_link_pass.argtypes = [i, i, _p(d), i, d, d, d, _p(d), u64, i, i, u32, u32, i, _p(d), _p(i)]
    L.or_class_pass.argtypes = [i, i, _p(d), i, i, i, d, d, d, _p(d), u64, i, i, u32, u32, i,
                                _p(d), _p(d)]
    L.or_class_pass.restype = i
    L.or_sweeps.argtypes = [i, i, i, _p(d), _p(d), _p(d), _p(d), _p(i), _p(d), i, u32, i, i, i,
                            u64, i, i, _p(i), _p(i)]
    L.or_replica_step.argtypes = [i, _p(i), _p(i), _p(d), _p(d), _p(d), _p(d), u64, i, u32, _p(C.c_longlong)]
    L.or_replica_run.argtypes = [i, i, i, _p(d), _p(d), _p(d), _p(d), _p(d), _p(i), _p(i), i, u32, u64, i, i,
                                 _p(d), _p(C.c_longlong)]
    L.or_llr_run.argtypes = [C.POINTER(RunParams), _p(d), C.POINTER(RunOut)]
    L.or_llr_run.restype = i
    L.or_rm_step.argtypes = [d, d, d, i, d]
    L.or_rm_step.restype = d
    L.or_ln_rho.argtypes = [_p(d), i, d, _p(d)]
    L.or_set_muca.argtypes = [_p(d), _p(d), i, d]
    L.or_muca_lnw.argtypes = [d]
    L.or_muca_lnw.restype = d
    L.or_reconstruct.argtypes = [_p(d), _p(d), i, d, d, _p(d), i, _p(d), _p(d), _p(d)]
    L.or_beta_c.argtypes = [_p(d), _p(d), i, d, d, d, d, d, d, _p(d), _p(d)]
    L.or_mlp_nparams.restype = i
    L.or_mlp_init.argtypes = [u64, _p(d)]
    L.or_mlp_forward.argtypes = [_p(d), _p(d), _p(d), i, _p(d), _p(d), _p(d)]
    L.or_mlp_loss_grad.argtypes = [_p(d), _p(d), _p(d), _p(d), i, _p(d)]
    L.or_mlp_loss_grad.restype = d
    L.or_mlp_adam.argtypes = [_p(d), _p(d), _p(d), _p(d), i, d, d, d, d]
    L.or_mlp_train.argtypes = [_p(d), _p(d), _p(d), _p(d), i, i, d, _p(d)]
    L.or_num_threads.restype = i


def _ptr(a, ctype):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(ctype))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _key(seed):
    return np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF], dtype=np.uint32)


def ctr1(attempt_pair=0, colour=0, kind=0, lattice_id=0):
    return (attempt_pair & 0xFF) | ((colour & 0xF) << 8) | ((kind & 0xF) << 12) | ((lattice_id & 0xFF) << 16)


# ---------------------------------------------------------------- wrappers
def philox(ctr, seed):
    """Philox4x32-10 of an (n, 4) uint32 counter array with key from seed."""
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    out = np.empty_like(ctr)
    key = _key(seed)
    lib().or_philox_batch(ctr.shape[0], _ptr(ctr, C.c_uint32), _ptr(key, C.c_uint32), _ptr(out, C.c_uint32))
    return out


def uniforms(words, u24=False):
    w = np.ascontiguousarray(words, dtype=np.uint32).ravel()
    u = np.empty(w.size)
    v = np.empty(w.size)
    lib().or_uniforms(w.size, _ptr(w, C.c_uint32), int(u24), _ptr(u, C.c_double), _ptr(v, C.c_double))
    return u, v


def neighbour(d, L, s, mu, step):
    return lib().or_neighbour(d, L, s, mu, step)


def energy(d, L, theta):
    th = _f64(theta)
    return lib().or_energy(d, L, _ptr(th, C.c_double))


def local_field(d, L, theta, mu, s):
    th = _f64(theta)
    c, sn = C.c_double(), C.c_double()
    lib().or_local_field(d, L, _ptr(th, C.c_double), mu, s, C.byref(c), C.byref(sn))
    return c.value, sn.value


def vonmises(n, kappa, seed, c1=0, c2=0, c3=0, u24=False):
    """n draws X ~ vM(kappa) with counters (i, c1, c2, c3); returns X, attempts, margin."""
    X = np.empty(n)
    att = np.empty(n, dtype=np.int32)
    mg = np.empty(n)
    lib().or_vonmises_batch(n, kappa, seed, c1, c2, c3, int(u24), _ptr(X, C.c_double),
                            _ptr(att, C.c_int), _ptr(mg, C.c_double))
    return X, att, mg


def link_draw(n, kappa, u_lo, u_hi, seed, c2=0, c3=0, u24=False):
    """n draws of the per-link restricted sampler, X ~ exp(kappa cos X) on
    cos X in [u_lo, u_hi], counters (i, colour 0, kind 0, lattice 0, c2, c3).
    Returns X and the stage that produced each draw (1, 2; 0 = none)."""
    X = np.empty(n)
    how = np.empty(n, dtype=np.int32)
    lib().or_link_draw_batch(n, kappa, u_lo, u_hi, seed, c2, c3, int(u24), _ptr(X, C.c_double),
                             _ptr(how, C.c_int))
    return X, how


def link_pass(d, L, theta, colour, a, lo, hi, E, seed, kind=KIND_SWEEP, lattice_id=0, sweep=0, interval=0,
              f32=False):
    """One heatbath pass of one colour under the per-link constraint (theta in
    place).  Returns (E, margin per class link, stage per class link)."""
    assert theta.dtype == np.float64 and theta.flags.c_contiguous
    e = C.c_double(E)
    V = L ** d
    mg = np.empty(V // 2)
    how = np.empty(V // 2, dtype=np.int32)
    lib().or_link_pass(d, L, _ptr(theta, C.c_double), colour, a, lo, hi, C.byref(e), seed, kind, lattice_id,
                       sweep, interval, int(f32), _ptr(mg, C.c_double), _ptr(how, C.c_int))
    return e.value, mg, how


def hot_start(d, L, n_chains, seed, lattice_id=0, f32=False):
    V = L ** d
    th = np.empty((n_chains, d, V))
    lib().or_hot_start(d, L, n_chains, seed, lattice_id, int(f32), _ptr(th, C.c_double))
    return th


def class_pass(d, L, theta, hb, colour, mode, a, lo, hi, E, seed, kind=KIND_SWEEP, lattice_id=0,
               sweep=0, interval=0, f32=False, want_margin=False):
    """One class pass on one chain (theta modified in place).  Returns (accept, E, dE, margin)."""
    assert theta.dtype == np.float64 and theta.flags.c_contiguous
    e = C.c_double(E)
    de = C.c_double(0.0)
    V = L ** d
    mg = np.empty(V // 2) if want_margin else None
    acc = lib().or_class_pass(d, L, _ptr(theta, C.c_double), int(hb), colour, mode, a, lo, hi,
                              C.byref(e), seed, kind, lattice_id, sweep, interval, int(f32),
                              _ptr(mg, C.c_double), C.byref(de))
    return acc, e.value, de.value, mg


def sweeps(d, L, theta, a, lo, hi, interval, E, n_sweeps, sweep0, mode=MODE_RESTRICTED,
           kind=KIND_SWEEP, do_or=True, seed=0, lattice_id=0, f32=False, order=SWEEP_GROUPED, use=None,
           chain=None, n_lattice_chains=None):
    """n_sweeps sweeps of every chain of theta (n_chains, d, V), in place.  Returns bits.
    order (with do_or): SWEEP_GROUPED, SWEEP_INTERLEAVED or SWEEP_STAGGERED;
    for the staggered order, chain (default 0, 1, ...) is each chain's index
    in its lattice and n_lattice_chains (default n_chains) the lattice's
    chain count: chains from ceil(n/2) on take their overrelaxation first.
    use: a library from build_variant instead of the oracle's own."""
    assert theta.dtype == np.float64 and theta.flags.c_contiguous
    nch = theta.shape[0]
    a, lo, hi = _f64(a), _f64(lo), _f64(hi)
    itv = np.ascontiguousarray(interval, dtype=np.int32)
    Earr = np.ascontiguousarray(E, dtype=np.float64).copy()
    bits = np.zeros((n_sweeps, nch), dtype=np.int32)
    per_chain = None
    if do_or and order == SWEEP_STAGGERED:
        ids = np.arange(nch) if chain is None else np.asarray(chain)
        n_lat = nch if n_lattice_chains is None else int(n_lattice_chains)
        per_chain = np.ascontiguousarray(np.where(ids < (n_lat + 1) // 2, 1, 3), dtype=np.int32)
    (use or lib()).or_sweeps(d, L, nch, _ptr(theta, C.c_double), _ptr(a, C.c_double), _ptr(lo, C.c_double),
                    _ptr(hi, C.c_double), _ptr(itv, C.c_int), _ptr(Earr, C.c_double), n_sweeps,
                    sweep0, mode, kind, (2 if order == SWEEP_INTERLEAVED else 1) if do_or else 0, seed,
                    lattice_id, int(f32), _ptr(bits, C.c_int), _ptr(per_chain, C.c_int))
    return Earr, bits


def llr_run(d, L, E_low, dE, a0, n_th, n_a, n_rm, seed, w=None, recompute_every=10,
            approach_cap=100000, replica_exchange=False, f32=False, lattice_id=0, eps=1e-4,
            theta=None, record_bits=False, per_link=False, order=SWEEP_GROUPED):
    """Algorithm 1 on every interval of one lattice.  Returns a dict of results.
    per_link: the restricted sweeps impose the restriction per link (Sec. 2.4)
    instead of rejecting whole colour classes.  order: of the class passes in
    a sweep (SWEEP_GROUPED, SWEEP_INTERLEAVED or SWEEP_STAGGERED; per-link
    sweeps stay grouped)."""
    E_low = _f64(E_low)
    n = E_low.size
    V = L ** d
    if w is None:
        w = 2.0 * dE if replica_exchange else dE
    p = RunParams(d, L, n, n_th, n_a, n_rm, recompute_every, approach_cap, int(replica_exchange),
                  int(f32), lattice_id, int(theta is None), seed, dE, w, eps, int(per_link),
                  {SWEEP_INTERLEAVED: 1, SWEEP_STAGGERED: 2}.get(order, 0))
    a = _f64(a0).copy() if np.ndim(a0) else np.full(n, float(a0))
    th = np.empty((n, d, V)) if theta is None else _f64(theta).copy()
    a_hist = np.zeros((n_rm + 1, n))
    E = np.zeros(n)
    conf = np.zeros(n, dtype=np.int32)
    conv = np.zeros(n, dtype=np.int32)
    convs = np.zeros(n, dtype=np.int64)
    ap = np.zeros(1, dtype=np.int64)
    nb = (approach_cap + recompute_every + n_rm * (n_th + n_a)) if record_bits else 0
    bits = np.zeros((nb, n), dtype=np.uint16) if record_bits else None
    sumE = np.zeros((n_rm, n))
    re = np.zeros(2, dtype=np.int64)
    out = RunOut(_ptr(a, C.c_double), _ptr(a_hist, C.c_double), _ptr(th, C.c_double),
                 _ptr(E, C.c_double), _ptr(conf, C.c_int), _ptr(conv, C.c_int),
                 _ptr(convs, C.c_longlong), _ptr(ap, C.c_longlong),
                 _ptr(bits, C.c_uint16) if record_bits else None, _ptr(sumE, C.c_double),
                 _ptr(re, C.c_longlong))
    rc = lib().or_llr_run(C.byref(p), _ptr(E_low, C.c_double), C.byref(out))
    if rc != 0:
        raise RuntimeError(f"oracle llr_run failed with status {rc}")
    res = dict(a=a, a_hist=a_hist, theta=th, E=E, conf=conf, conv_iter=conv, conv_sweeps=convs,
               approach_sweeps=int(ap[0]), sumE_hist=sumE, re=re, w=w)
    if record_bits:
        res["bits"] = bits[: int(ap[0]) + n_rm * (n_th + n_a)]
    return res


def replica_step(conf, itv, E, a, lo, hi, seed, t, lattice_id=0, re_acc=None, use=None):
    """Replica exchange after sweep t (Sec. 2.5) on n intervals: conf
    (interval -> chain) and itv (chain -> interval), int32 arrays, are updated
    in place; E per chain; a, lo, hi per interval; re_acc (int64[2], optional)
    accumulates [proposed, accepted]."""
    for x in (conf, itv):
        assert x.dtype == np.int32 and x.flags.c_contiguous
    E, a, lo, hi = _f64(E), _f64(a), _f64(lo), _f64(hi)
    if re_acc is not None:
        assert re_acc.dtype == np.int64
    (use or lib()).or_replica_step(a.size, _ptr(conf, C.c_int), _ptr(itv, C.c_int), _ptr(E, C.c_double),
                                   _ptr(a, C.c_double), _ptr(lo, C.c_double), _ptr(hi, C.c_double), seed,
                                   lattice_id, t, _ptr(re_acc, C.c_longlong))


def replica_run(d, L, theta, a, lo, hi, E, conf, itv, n_sweeps, sweep0, seed, lattice_id=0,
                order=SWEEP_GROUPED, re_acc=None, use=None):
    """n_sweeps of (restricted sweep of every chain at the coupling of the
    interval it serves, then replica_step) at fixed a.  theta (n, d, V), E,
    conf, itv are updated in place.  Returns the energies visited by each
    interval after every exchange, (n_sweeps, n)."""
    assert theta.dtype == np.float64 and theta.flags.c_contiguous
    for x in (conf, itv):
        assert x.dtype == np.int32 and x.flags.c_contiguous
    assert E.dtype == np.float64 and E.flags.c_contiguous
    a, lo, hi = _f64(a), _f64(lo), _f64(hi)
    n = a.size
    vis = np.empty((n_sweeps, n))
    (use or lib()).or_replica_run(d, L, n, _ptr(theta, C.c_double), _ptr(a, C.c_double), _ptr(lo, C.c_double),
                                  _ptr(hi, C.c_double), _ptr(E, C.c_double), _ptr(conf, C.c_int),
                                  _ptr(itv, C.c_int), n_sweeps, sweep0, seed, lattice_id,
                                  1 if order == SWEEP_INTERLEAVED else 0, _ptr(vis, C.c_double),
                                  _ptr(re_acc, C.c_longlong))
    return vis


def rm_step(a, mean, centre, n, w):
    """One Robbins-Monro update of eq. (kk21) (Algorithm 1 sign)."""
    return lib().or_rm_step(float(a), float(mean), float(centre), int(n), float(w))


def ln_rho(a, s):
    a = _f64(a)
    out = np.empty_like(a)
    lib().or_ln_rho(_ptr(a, C.c_double), a.size, s, _ptr(out, C.c_double))
    return out


def reconstruct(centres, a, s, six_v, beta):
    c, a, b = _f64(centres), _f64(a), _f64(beta)
    lr = np.empty(a.size)
    u = np.empty(b.size)
    cv = np.empty(b.size)
    lib().or_reconstruct(_ptr(c, C.c_double), _ptr(a, C.c_double), a.size, s, six_v,
                         _ptr(b, C.c_double), b.size, _ptr(lr, C.c_double), _ptr(u, C.c_double),
                         _ptr(cv, C.c_double))
    return lr, u, cv


def beta_c(centres, a, s, six_v, blo, bhi, h=1e-5, tol=1e-9):
    c, a = _f64(centres), _f64(a)
    bc, pk = C.c_double(), C.c_double()
    lib().or_beta_c(_ptr(c, C.c_double), _ptr(a, C.c_double), a.size, s, six_v, blo, bhi, h, tol,
                    C.byref(bc), C.byref(pk))
    return bc.value, pk.value


# --------------------------------------------- analysis of repeated runs
def log_rho_tilde(centres, a, s, E):
    """ln rho~(E) of eq. (rhoguess) relative to the first centre: in interval k
    ln rho~ = L_k - a_k (E - c_k), with L_k from the trapezium recursion."""
    c, a, E = _f64(centres), _f64(a), np.atleast_1d(_f64(E))
    L = ln_rho(a, s)
    out = np.full(E.size, -np.inf)
    lo, hi = c[0] - 0.5 * s, c[-1] + 0.5 * s
    for i, e in enumerate(E):
        if lo <= e <= hi:
            k = min(int(np.floor((e - lo) / s)), c.size - 1)
            out[i] = L[k] - a[k] * (e - c[k])
    return out


def prob_density(centres, a, s, beta, E):
    """ln P_beta(E) = ln rho~(E) + beta E - ln Z (Sec. 3.4), Z the integral of
    rho~ e^{beta E} over the covered range, interval by interval:
    int_{c-s/2}^{c+s/2} e^{L - a (E - c) + beta E} dE = e^{L + beta c} s sinh(x)/x,
    x = (beta - a) s / 2."""
    c, a = _f64(centres), _f64(a)
    L = ln_rho(a, s)
    x = (beta - a) * 0.5 * s
    ax = np.abs(x)
    with np.errstate(divide="ignore", invalid="ignore"):
        lsh = np.where(ax < 1e-6, ax * ax / 6.0, np.log(np.sinh(np.minimum(ax, 700.0)) / np.maximum(ax, 1e-300)))
    lsh = np.where(ax > 700.0, ax - np.log(2.0 * ax), lsh)
    t = L + beta * c + lsh
    m = t.max()
    lnz = m + np.log(s * np.sum(np.exp(t - m)))
    lr = log_rho_tilde(c, a, s, E)
    return lr + beta * np.atleast_1d(_f64(E)) - lnz


def prob_peaks(centres, a, s, beta):
    """Interior local maxima of ln P_beta(E), found by comparing its values at
    the breakpoints (the interval edges), between which it is linear: edge k
    (between intervals k and k+1) is a maximum iff its value exceeds the
    previous edge's and is not below the next one's."""
    c, a = _f64(centres), _f64(a)
    edges = np.concatenate([[c[0] - 0.5 * s], c + 0.5 * s])
    v = prob_density(c, a, s, beta, edges)
    pk = [k for k in range(1, edges.size - 1) if v[k] > v[k - 1] and v[k] >= v[k + 1]]
    return edges[pk], v[pk]


def bootstrap_indices(n_runs, n_boot, seed):
    """Draw j of sample b: floor(n_runs w / 2^32), w the first Philox word of
    counter (j, kind 5 << 12, b, 0)."""
    j, b = np.meshgrid(np.arange(n_runs), np.arange(n_boot))
    ctr = np.zeros((n_boot * n_runs, 4), dtype=np.uint32)
    ctr[:, 0] = j.ravel()
    ctr[:, 1] = ctr1(kind=KIND_BOOT)
    ctr[:, 2] = b.ravel()
    w = philox(ctr, seed)[:, 0].astype(np.uint64)
    return ((w * np.uint64(n_runs)) >> np.uint64(32)).astype(np.int64).reshape(n_boot, n_runs)


def bootstrap(centres, a_runs, s, six_v, blo, bhi, n_boot, seed, h=1e-5, tol=1e-9):
    """beta_c and the C_V peak of each bootstrap sample: the mean a_k of the
    drawn runs (summed in draw order), reconstructed by beta_c()."""
    ar = np.atleast_2d(_f64(a_runs))
    idx = bootstrap_indices(ar.shape[0], n_boot, seed)
    bc, pk = np.empty(n_boot), np.empty(n_boot)
    for b in range(n_boot):
        acc = np.zeros(ar.shape[1])
        for j in idx[b]:
            acc = acc + ar[j]
        bc[b], pk[b] = beta_c(centres, acc / ar.shape[0], s, six_v, blo, bhi, h, tol)
    return bc, pk


# ---------------------------- observables from double brackets (Sec. 2.3)
def adjoint(d, L, theta):
    """sum_P cos(2 theta_P) of one chain."""
    th = _f64(theta)
    return lib().or_adjoint(d, L, _ptr(th, C.c_double))


def obs_reconstruct(centres, a, s, E, B, beta):
    """Eqs. (l9)-(l10) with the interval centres as reference energies:
    <B> = sum_k rho~(c_k) e^{beta c_k} <<B e^{(beta-a_k)(E-c_k)}>>_k
        / sum_k rho~(c_k) e^{beta c_k} <<e^{(beta-a_k)(E-c_k)}>>_k,
    <<.>>_k the mean over the samples (rows) of column k."""
    c, a = _f64(centres), _f64(a)
    E, B = np.atleast_2d(_f64(E)), np.atleast_2d(_f64(B))
    lr = ln_rho(a, s)
    out = []
    for b in np.atleast_1d(beta):
        x = (b - a)[None, :] * (E - c[None, :])
        xm = x.max(axis=0)
        w = np.exp(x - xm[None, :])
        D = w.mean(axis=0)
        N = (w * B).mean(axis=0)
        lw = lr + b * c + xm + np.log(D)
        p = np.exp(lw - lw.max())
        out.append(np.sum(p * N / D) / np.sum(p))
    return np.array(out)


# ------------------------------------ multicanonical sampling (Sec. 2.6)
def set_muca(centres, a, s):
    """Weight W = 1/rho~ for MODE_MUCA passes and sweeps (the proposal coupling
    is the per-chain a passed to those calls)."""
    c, a = _f64(centres), _f64(a)
    lib().or_set_muca(_ptr(c, C.c_double), _ptr(a, C.c_double), a.size, s)


def muca_lnw(E):
    return np.array([lib().or_muca_lnw(float(e)) for e in np.atleast_1d(E)])


def muca_reweight(E, centres, a, s, six_v, beta):
    """Eq. (4.7): <O>_beta = <O e^{beta E}/W(E)>_W / <e^{beta E}/W(E)>_W for
    O = E, (E - <E>)^2; returns <u> = <E>/(6V), C_V = Var(E)/(6V)."""
    E = np.ravel(_f64(E))
    set_muca(centres, a, s)
    lw = muca_lnw(E)
    u, cv = [], []
    for b in np.atleast_1d(beta):
        t = b * E - lw
        w = np.exp(t - t.max())
        mu = np.sum(w * E) / np.sum(w)
        u.append(mu / six_v)
        cv.append(np.sum(w * (E - mu) ** 2) / np.sum(w) / six_v)
    return np.array(u), np.array(cv)


def fss_fit(L, y, sigma, powers):
    """Weighted least squares for y(L) = sum_j p_j L^powers_j (the finite-size
    forms of Sec. 3.4) with numpy's lstsq; errors sqrt(diag((A^T A)^-1)) of the
    weighted design matrix A, chi2_red = |A p - y/sigma|^2 / (m - n_par)."""
    L, y, sg, pw = _f64(L), _f64(y), _f64(sigma), _f64(powers)
    A = L[:, None] ** pw[None, :] / sg[:, None]
    col = np.sqrt(np.sum(A * A, axis=0))
    As = A / col
    p, _, _, _ = np.linalg.lstsq(As, y / sg, rcond=None)
    r = As @ p - y / sg
    cov = np.linalg.inv(As.T @ As)
    return p / col, np.sqrt(np.diag(cov)) / col, float(r @ r) / (L.size - pw.size)


def mlp_init(seed):
    w = np.empty(N_PARAMS)
    lib().or_mlp_init(seed, _ptr(w, C.c_double))
    return w


def mlp_forward(w, u, invL, want_hidden=False):
    w, u, invL = _f64(w), _f64(u), _f64(invL)
    n = u.size
    a = np.empty(n)
    h1 = np.empty((n, 64)) if want_hidden else None
    h2 = np.empty((n, 64)) if want_hidden else None
    lib().or_mlp_forward(_ptr(w, C.c_double), _ptr(u, C.c_double), _ptr(invL, C.c_double), n,
                         _ptr(a, C.c_double), _ptr(h1, C.c_double), _ptr(h2, C.c_double))
    return (a, h1, h2) if want_hidden else a


def mlp_loss_grad(w, u, invL, a):
    w, u, invL, a = _f64(w), _f64(u), _f64(invL), _f64(a)
    g = np.empty(N_PARAMS)
    loss = lib().or_mlp_loss_grad(_ptr(w, C.c_double), _ptr(u, C.c_double), _ptr(invL, C.c_double),
                                  _ptr(a, C.c_double), u.size, _ptr(g, C.c_double))
    return loss, g


def mlp_adam(w, m, v, g, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    for x in (w, m, v):
        assert x.dtype == np.float64 and x.flags.c_contiguous
    g = _f64(g)
    lib().or_mlp_adam(_ptr(w, C.c_double), _ptr(m, C.c_double), _ptr(v, C.c_double),
                      _ptr(g, C.c_double), t, lr, b1, b2, eps)


def mlp_train(w, u, invL, a, epochs, lr):
    w = _f64(w).copy()
    u, invL, a = _f64(u), _f64(invL), _f64(a)
    hist = np.empty(epochs)
    lib().or_mlp_train(_ptr(w, C.c_double), _ptr(u, C.c_double), _ptr(invL, C.c_double),
                       _ptr(a, C.c_double), u.size, epochs, lr, _ptr(hist, C.c_double))
    return w, hist


def num_threads():
    return lib().or_num_threads()
