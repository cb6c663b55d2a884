"""Thin ctypes binding of libllr.so (include/llr.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  PyTorch provides the device memory of the link state and the
stream.  Importing works without a GPU; creating a context needs the built
library and a HIP device and raises otherwise (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libllr.so")

OK, WARN_NOT_CONVERGED = 0, 1
FP64, FP32 = 0, 1
MODE_RESTRICTED, MODE_APPROACH, MODE_FREE, MODE_MUCA, MODE_LINK = 0, 1, 2, 3, 4
SWEEP_GROUPED, SWEEP_INTERLEAVED, SWEEP_STAGGERED = 0, 1, 2
N_PARAMS = 4417

_lib = None


class LLRError(RuntimeError):
    pass


class LLRNumericError(LLRError):
    """LLR_ENUMERIC: a chain failed a health test (Context.health)."""


class Rates(C.Structure):
    _fields_ = [("sweeps", C.c_longlong), ("hb_class_passes", C.c_longlong), ("hb_class_accepts", C.c_longlong),
                ("or_class_passes", C.c_longlong), ("or_class_relabelled", C.c_longlong),
                ("re_proposals", C.c_longlong), ("re_accepts", C.c_longlong), ("link_updates", C.c_double),
                ("seconds", C.c_double), ("link_updates_per_s", C.c_double), ("hb_acceptance", C.c_double),
                ("or_acceptance", C.c_double), ("re_acceptance", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Params(C.Structure):
    _fields_ = [("n_th", C.c_int), ("n_a", C.c_int), ("n_rm", C.c_int), ("seed", C.c_uint64),
                ("replica_exchange", C.c_int), ("overlap", C.c_double), ("recompute_every", C.c_int),
                ("eps", C.c_double), ("approach_cap", C.c_int)]


def _p(t):
    return C.POINTER(t)


_SIGS = {
    "llr_create": [_p(C.c_void_p), C.c_int, C.c_void_p, C.c_int],
    "llr_set_params": [C.c_void_p, _p(Params)],
    "llr_add_lattice": [C.c_void_p, C.c_int, C.c_int, _p(C.c_double), C.c_double, _p(C.c_int)],
    "llr_state_bytes": [C.c_void_p, _p(C.c_size_t)],
    "llr_bind_state": [C.c_void_p, C.c_void_p, C.c_size_t],
    "llr_set_a": [C.c_void_p, C.c_int, _p(C.c_double)],
    "llr_hot_start": [C.c_void_p],
    "llr_import_state": [C.c_void_p, C.c_int, C.c_void_p],
    "llr_export_state": [C.c_void_p, C.c_int, C.c_void_p],
    "llr_approach": [C.c_void_p, _p(C.c_longlong)],
    "llr_approach_begin": [C.c_void_p],
    "llr_approach_continue": [C.c_void_p, C.c_longlong, _p(C.c_longlong), _p(C.c_int)],
    "llr_run": [C.c_void_p],
    "llr_rm_begin": [C.c_void_p],
    "llr_rm_step": [C.c_void_p, C.c_int],
    "llr_set_restriction": [C.c_void_p, C.c_int],
    "llr_get_a": [C.c_void_p, C.c_int, _p(C.c_double), _p(C.c_int), _p(C.c_longlong)],
    "llr_get_history": [C.c_void_p, C.c_int, _p(C.c_double)],
    "llr_get_energy": [C.c_void_p, C.c_int, _p(C.c_double), _p(C.c_int)],
    "llr_get_ln_rho": [C.c_void_p, C.c_int, _p(C.c_double), _p(C.c_double)],
    "llr_sweeps": [C.c_void_p, C.c_int, C.c_longlong, C.c_int, _p(C.c_uint16)],
    "llr_recompute_energy": [C.c_void_p],
    "llr_class_pass": [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_longlong],
    "llr_autotune": [C.c_void_p, _p(C.c_int), _p(C.c_int)],
    "llr_set_tiles": [C.c_void_p, C.c_int, C.c_int],
    "llr_set_order": [C.c_void_p, C.c_int],
    "llr_set_sweep_order": [C.c_void_p, C.c_int],
    "llr_set_graphs": [C.c_void_p, C.c_int],
    "llr_enable_bits_log": [C.c_void_p, C.c_longlong],
    "llr_get_bits_log": [C.c_void_p, _p(C.c_uint16), _p(C.c_longlong)],
    "llr_stats": [C.c_void_p, _p(C.c_longlong), _p(C.c_longlong), _p(C.c_longlong), _p(C.c_longlong)],
    "llr_get_rates": [C.c_void_p, _p(Rates)],
    "llr_health": [C.c_void_p, _p(C.c_uint32), _p(C.c_double), C.c_int],
    "llr_link_stats": [C.c_void_p, _p(C.c_longlong), _p(C.c_longlong)],
    "llr_checkpoint": [C.c_void_p, C.c_char_p],
    "llr_restore": [C.c_void_p, C.c_char_p],
    "llr_checkpoint_info": [C.c_char_p, _p(C.c_int), _p(C.c_int), _p(C.c_int), _p(C.c_int), _p(C.c_double),
                            _p(C.c_double), _p(Params)],
    "llr_set_timing": [C.c_void_p, C.c_int],
    "llr_get_timing": [C.c_void_p, _p(C.c_double), _p(C.c_longlong), _p(C.c_double), _p(C.c_longlong),
                       _p(C.c_double), _p(C.c_longlong)],
    "llr_test_philox": [C.c_void_p, C.c_long, _p(C.c_uint32), C.c_uint64, _p(C.c_uint32)],
    "llr_test_vonmises": [C.c_void_p, C.c_long, C.c_double, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32,
                          _p(C.c_double), _p(C.c_int)],
    "llr_reconstruct": [C.c_void_p, _p(C.c_double), _p(C.c_double), C.c_int, C.c_double, C.c_double,
                        _p(C.c_double), C.c_int, _p(C.c_double), _p(C.c_double), _p(C.c_double)],
    "llr_beta_c": [C.c_void_p, _p(C.c_double), _p(C.c_double), C.c_int, C.c_double, C.c_double, C.c_double,
                   C.c_double, C.c_double, C.c_double, _p(C.c_double), _p(C.c_double)],
    "llr_beta_c_noalloc": [C.c_void_p, _p(C.c_double), _p(C.c_double), C.c_int, C.c_double, C.c_double,
                           C.c_double, C.c_double, C.c_double, C.c_double, _p(C.c_double), _p(C.c_double)],
    "llr_prob_density": [C.c_void_p, _p(C.c_double), _p(C.c_double), C.c_int, C.c_double, C.c_double,
                         _p(C.c_double), C.c_int, _p(C.c_double)],
    "llr_prob_peaks": [C.c_void_p, _p(C.c_double), _p(C.c_double), C.c_int, C.c_double, C.c_double, C.c_int,
                       _p(C.c_double), _p(C.c_double), _p(C.c_int)],
    "llr_bootstrap": [C.c_void_p, _p(C.c_double), _p(C.c_double), C.c_int, C.c_int, C.c_double, C.c_double,
                      C.c_double, C.c_double, C.c_double, C.c_double, C.c_int, C.c_uint64, _p(C.c_double),
                      _p(C.c_double)],
    "llr_fss_fit": [_p(C.c_double), _p(C.c_double), _p(C.c_double), C.c_int, _p(C.c_double), C.c_int,
                    _p(C.c_double), _p(C.c_double), _p(C.c_double)],
    "llr_observables": [C.c_void_p, C.c_int, C.c_int, C.c_longlong, _p(C.c_double), _p(C.c_double)],
    "llr_obs_reconstruct": [C.c_void_p, _p(C.c_double), _p(C.c_double), C.c_int, C.c_double, _p(C.c_double),
                            _p(C.c_double), C.c_int, _p(C.c_double), C.c_int, _p(C.c_double)],
    "llr_muca_begin": [C.c_void_p, _p(C.c_double)],
    "llr_muca_sweeps": [C.c_void_p, C.c_int, C.c_longlong, _p(C.c_double)],
    "llr_muca_reweight": [C.c_void_p, _p(C.c_double), C.c_long, _p(C.c_double), _p(C.c_double), C.c_int,
                          C.c_double, C.c_double, _p(C.c_double), C.c_int, _p(C.c_double), _p(C.c_double)],
    "llr_mlp_init": [C.c_void_p, C.c_uint64, _p(C.c_float)],
    "llr_mlp_predict": [C.c_void_p, _p(C.c_float), _p(C.c_float), _p(C.c_float), C.c_int, C.c_int,
                        _p(C.c_double)],
    "llr_mlp_warm_start": [C.c_void_p, C.c_int, _p(C.c_float), C.c_int, C.c_double, C.c_double, _p(C.c_double),
                           _p(C.c_int)],
    "llr_mlp_loss_grad": [C.c_void_p, _p(C.c_float), _p(C.c_float), _p(C.c_float), _p(C.c_double), C.c_int,
                          C.c_int, _p(C.c_float), _p(C.c_double)],
    "llr_mlp_train": [C.c_void_p, _p(C.c_float), _p(C.c_float), _p(C.c_float), _p(C.c_double), C.c_int, C.c_int,
                      C.c_float, C.c_int, _p(C.c_double)],
}


def lib():
    """Load libllr.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise LLRError(f"{LIB_PATH} is missing: build it with paper_1509_08391_amd/build.py")
        L = C.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.llr_last_error.restype = C.c_char_p
        L.llr_destroy.argtypes = [C.c_void_p]
        L.llr_destroy.restype = None
        _lib = L
    return _lib


ENUMERIC = -6


def _check(st, allow_warn=False):
    if st < 0 or (st > 0 and not allow_warn):
        cls = LLRNumericError if st == ENUMERIC else LLRError
        raise cls(f"llr status {st}: {lib().llr_last_error().decode()}")
    return st


def _arr(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a, ctype):
    return None if a is None else a.ctypes.data_as(C.POINTER(ctype))


def _stream_handle(stream):
    if stream is None:
        return None
    return C.c_void_p(int(stream.cuda_stream))


class Context:
    """One LLR context on one GPU.  Lattices are added first, then the link
    state is allocated with torch and bound; all heavy work runs in HIP."""

    def __init__(self, precision=FP32, device=0, stream=None):
        import torch
        self.torch = torch
        self.device = device
        self.precision = precision
        self.dtype = torch.float32 if precision == FP32 else torch.float64
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        h = C.c_void_p()
        _check(lib().llr_create(C.byref(h), device, _stream_handle(self.stream), precision))
        self.h = h
        self.lattices = []     # (L, n, E_low, dE)
        self.state = None

    def close(self):
        if getattr(self, "h", None):
            lib().llr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- configuration
    def set_params(self, n_th=100, n_a=100, n_rm=20, seed=1509083910, replica_exchange=False, overlap=1.0,
                   recompute_every=10, eps=1e-4, approach_cap=100000):
        p = Params(n_th, n_a, n_rm, seed, int(replica_exchange), overlap, recompute_every, eps, approach_cap)
        _check(lib().llr_set_params(self.h, C.byref(p)))
        self.params = p

    def add_lattice(self, L, E_low, dE):
        E_low = _arr(E_low, np.float64)
        lid = C.c_int()
        _check(lib().llr_add_lattice(self.h, L, E_low.size, _ptr(E_low, C.c_double), dE, C.byref(lid)))
        self.lattices.append((L, E_low.size, E_low.copy(), dE))
        return lid.value

    def bind_state(self):
        """Allocate the link state with torch (caller-owned) and bind it."""
        nb = C.c_size_t()
        _check(lib().llr_state_bytes(self.h, C.byref(nb)))
        esz = 4 if self.precision == FP32 else 8
        self.state = self.torch.empty(nb.value // esz, dtype=self.dtype, device=f"cuda:{self.device}")
        _check(lib().llr_bind_state(self.h, C.c_void_p(self.state.data_ptr()), nb.value))
        return self.state

    def set_a(self, lattice_id, a):
        n = self.lattices[lattice_id][1]
        a = _arr(np.broadcast_to(np.asarray(a, dtype=np.float64), (n,)), np.float64)
        _check(lib().llr_set_a(self.h, lattice_id, _ptr(a, C.c_double)))

    # ---- state
    def hot_start(self):
        _check(lib().llr_hot_start(self.h))

    def import_state(self, lattice_id, theta):
        """theta: torch tensor on the device, (n, 4, V) canonical, context dtype."""
        t = theta.to(device=f"cuda:{self.device}", dtype=self.dtype).contiguous()
        _check(lib().llr_import_state(self.h, lattice_id, C.c_void_p(t.data_ptr())))

    def export_state(self, lattice_id):
        L, n = self.lattices[lattice_id][:2]
        out = self.torch.empty((n, 4, L ** 4), dtype=self.dtype, device=f"cuda:{self.device}")
        _check(lib().llr_export_state(self.h, lattice_id, C.c_void_p(out.data_ptr())))
        return out

    # ---- Algorithm 1
    def approach(self):
        s = np.zeros(len(self.lattices), dtype=np.int64)
        _check(lib().llr_approach(self.h, _ptr(s, C.c_longlong)))
        return s

    def approach_begin(self):
        _check(lib().llr_approach_begin(self.h))

    def approach_continue(self, max_sweeps):
        s = np.zeros(len(self.lattices), dtype=np.int64)
        done = C.c_int()
        _check(lib().llr_approach_continue(self.h, max_sweeps, _ptr(s, C.c_longlong), C.byref(done)))
        return s, bool(done.value)

    def run(self):
        return _check(lib().llr_run(self.h), allow_warn=True)

    def rm_begin(self):
        _check(lib().llr_rm_begin(self.h))

    def rm_step(self, iterations=1):
        return _check(lib().llr_rm_step(self.h, iterations), allow_warn=True)

    def get_a(self, lattice_id):
        n = self.lattices[lattice_id][1]
        a = np.empty(n)
        it = np.empty(n, dtype=np.int32)
        sw = np.empty(n, dtype=np.int64)
        _check(lib().llr_get_a(self.h, lattice_id, _ptr(a, C.c_double), _ptr(it, C.c_int), _ptr(sw, C.c_longlong)))
        return a, it, sw

    def get_history(self, lattice_id):
        n = self.lattices[lattice_id][1]
        h = np.empty((self.params.n_rm + 1, n))
        _check(lib().llr_get_history(self.h, lattice_id, _ptr(h, C.c_double)))
        return h

    def get_energy(self, lattice_id):
        n = self.lattices[lattice_id][1]
        E = np.empty(n)
        conf = np.empty(n, dtype=np.int32)
        _check(lib().llr_get_energy(self.h, lattice_id, _ptr(E, C.c_double), _ptr(conf, C.c_int)))
        return E, conf

    def get_ln_rho(self, lattice_id):
        n = self.lattices[lattice_id][1]
        c = np.empty(n)
        lr = np.empty(n)
        _check(lib().llr_get_ln_rho(self.h, lattice_id, _ptr(c, C.c_double), _ptr(lr, C.c_double)))
        return c, lr

    # ---- hooks
    def sweeps(self, n_sweeps, sweep0=0, mode=MODE_RESTRICTED, want_bits=True):
        nch = sum(x[1] for x in self.lattices)
        bits = np.zeros((n_sweeps, nch), dtype=np.uint16) if want_bits else None
        _check(lib().llr_sweeps(self.h, n_sweeps, sweep0, mode, _ptr(bits, C.c_uint16)))
        return bits

    def autotune(self):
        hb, orr = C.c_int(), C.c_int()
        _check(lib().llr_autotune(self.h, C.byref(hb), C.byref(orr)))
        return hb.value, orr.value

    def set_graphs(self, on):
        _check(lib().llr_set_graphs(self.h, int(on)))

    def set_restriction(self, per_link):
        """Restricted sweeps of run / rm_step and the measurements: per link
        (True) or class-wise rejection (False, the default)."""
        _check(lib().llr_set_restriction(self.h, int(per_link)))

    def set_order(self, serpentine):
        _check(lib().llr_set_order(self.h, int(serpentine)))

    def set_sweep_order(self, order):
        """SWEEP_GROUPED (heatbath of every colour, then overrelaxation of
        every colour), SWEEP_INTERLEAVED (heatbath then overrelaxation per
        colour, fused in one launch) or SWEEP_STAGGERED (grouped on the first
        half of each lattice's chains, overrelaxation first on the others,
        the two halves on two streams)."""
        _check(lib().llr_set_sweep_order(self.h, int(order)))

    def set_tiles(self, hb_lpt, or_lpt):
        _check(lib().llr_set_tiles(self.h, hb_lpt, or_lpt))

    def class_pass(self, heatbath, colour, mode=MODE_RESTRICTED, sweep_index=0):
        _check(lib().llr_class_pass(self.h, int(heatbath), colour, mode, sweep_index))

    def recompute_energy(self):
        _check(lib().llr_recompute_energy(self.h))

    def enable_bits_log(self, max_rows):
        _check(lib().llr_enable_bits_log(self.h, max_rows))
        self._bits_max = max_rows

    def get_bits_log(self):
        nch = sum(x[1] for x in self.lattices)
        bits = np.zeros((self._bits_max, nch), dtype=np.uint16)
        rows = C.c_longlong()
        _check(lib().llr_get_bits_log(self.h, _ptr(bits, C.c_uint16), C.byref(rows)))
        return bits[: rows.value]

    def stats(self):
        nch = sum(x[1] for x in self.lattices)
        hp = np.zeros(nch, dtype=np.int64)
        ha = np.zeros(nch, dtype=np.int64)
        rp, ra = C.c_longlong(), C.c_longlong()
        _check(lib().llr_stats(self.h, _ptr(hp, C.c_longlong), _ptr(ha, C.c_longlong), C.byref(rp), C.byref(ra)))
        return hp, ha, rp.value, ra.value

    def rates(self):
        """Work done and rates since creation (llr_get_rates) as a dict."""
        r = Rates()
        _check(lib().llr_get_rates(self.h, C.byref(r)))
        return r.as_dict()

    def health(self, clear=False):
        """Per chain: health flags (1 non-finite angle, 2 drift beyond the
        bound, 4 E outside the restriction) and the largest drift seen at a
        recompute; clear resets both."""
        nch = sum(x[1] for x in self.lattices)
        f = np.zeros(nch, dtype=np.uint32)
        d = np.zeros(nch, dtype=np.float64)
        _check(lib().llr_health(self.h, _ptr(f, C.c_uint32), _ptr(d, C.c_double), 1 if clear else 0))
        return f, d

    # ---- checkpoints
    def checkpoint(self, path):
        """Save the whole state of Algorithm 1 (angles, bits, E, a_k, counters,
        chain <-> interval labels, history) to path."""
        _check(lib().llr_checkpoint(self.h, os.fsencode(path)))

    def restore(self, path):
        """Load a checkpoint written for the same precision and lattice set
        into this context (state bound)."""
        _check(lib().llr_restore(self.h, os.fsencode(path)))
        self.params = checkpoint_info(path)["params"]

    @classmethod
    def from_checkpoint(cls, path, device=0, stream=None):
        """A new context with the checkpoint's precision, lattices and
        parameters, its state allocated, bound and restored."""
        info = checkpoint_info(path)
        ctx = cls(precision=info["precision"], device=device, stream=stream)
        _check(lib().llr_set_params(ctx.h, C.byref(info["params"])))
        ctx.params = info["params"]
        for L, E_low, dE in info["lattices"]:
            ctx.add_lattice(L, E_low, dE)
        ctx.bind_state()
        ctx.restore(path)
        return ctx

    def link_stats(self):
        """Per chain: links re-drawn under the per-link constraint and, of
        those, draws of the arc sampler (cumulative)."""
        nch = sum(x[1] for x in self.lattices)
        fx = np.zeros(nch, dtype=np.int64)
        ar = np.zeros(nch, dtype=np.int64)
        _check(lib().llr_link_stats(self.h, _ptr(fx, C.c_longlong), _ptr(ar, C.c_longlong)))
        return fx, ar

    def set_timing(self, on):
        _check(lib().llr_set_timing(self.h, int(on)))

    def get_timing(self):
        v = [C.c_double(), C.c_longlong(), C.c_double(), C.c_longlong(), C.c_double(), C.c_longlong()]
        _check(lib().llr_get_timing(self.h, *[C.byref(x) for x in v]))
        return dict(hb_ms=v[0].value, hb_n=v[1].value, or_ms=v[2].value, or_n=v[3].value,
                    energy_ms=v[4].value, energy_n=v[5].value)

    def test_philox(self, ctr, seed):
        ctr = _arr(ctr, np.uint32).reshape(-1, 4)
        out = np.empty_like(ctr)
        _check(lib().llr_test_philox(self.h, ctr.shape[0], _ptr(ctr, C.c_uint32), seed, _ptr(out, C.c_uint32)))
        return out

    def test_vonmises(self, n, kappa, seed, c1=0, c2=0, c3=0):
        X = np.empty(n)
        att = np.empty(n, dtype=np.int32)
        _check(lib().llr_test_vonmises(self.h, n, kappa, seed, c1, c2, c3, _ptr(X, C.c_double), _ptr(att, C.c_int)))
        return X, att

    # ---- reconstruction
    def reconstruct(self, centres, a, s, six_v, beta):
        c, a, b = _arr(centres, np.float64), _arr(a, np.float64), _arr(np.atleast_1d(beta), np.float64)
        lr, u, cv = np.empty(a.size), np.empty(b.size), np.empty(b.size)
        _check(lib().llr_reconstruct(self.h, _ptr(c, C.c_double), _ptr(a, C.c_double), a.size, s, six_v,
                                     _ptr(b, C.c_double), b.size, _ptr(lr, C.c_double), _ptr(u, C.c_double),
                                     _ptr(cv, C.c_double)))
        return lr, u, cv

    def beta_c(self, centres, a, s, six_v, blo, bhi, h=1e-5, tol=1e-9):
        c, a = _arr(centres, np.float64), _arr(a, np.float64)
        bc, pk = C.c_double(), C.c_double()
        _check(lib().llr_beta_c(self.h, _ptr(c, C.c_double), _ptr(a, C.c_double), a.size, s, six_v, blo, bhi, h,
                                tol, C.byref(bc), C.byref(pk)))
        return bc.value, pk.value

    def beta_c_noalloc(self, centres, a, s, six_v, blo, bhi, h=1e-5, tol=1e-9):
        """beta_c through the allocation-free entry point (fixed 1 MiB device
        buffer per GPU; see llr_beta_c_noalloc)."""
        c, a = _arr(centres, np.float64), _arr(a, np.float64)
        bc, pk = C.c_double(), C.c_double()
        _check(lib().llr_beta_c_noalloc(self.h, _ptr(c, C.c_double), _ptr(a, C.c_double), a.size, s, six_v, blo, bhi,
                                        h, tol, C.byref(bc), C.byref(pk)))
        return bc.value, pk.value

    def prob_density(self, centres, a, s, beta, E):
        """ln P_beta(E) of the piecewise-exponential density of states."""
        c, a, E = _arr(centres, np.float64), _arr(a, np.float64), _arr(np.atleast_1d(E), np.float64)
        out = np.empty(E.size)
        _check(lib().llr_prob_density(self.h, _ptr(c, C.c_double), _ptr(a, C.c_double), a.size, s, beta,
                                      _ptr(E, C.c_double), E.size, _ptr(out, C.c_double)))
        return out

    def prob_peaks(self, centres, a, s, beta, max_peaks=64):
        """Interior maxima of P_beta(E): (energies, ln P) in ascending E."""
        c, a = _arr(centres, np.float64), _arr(a, np.float64)
        Ep, lp, nf = np.empty(max_peaks), np.empty(max_peaks), C.c_int()
        _check(lib().llr_prob_peaks(self.h, _ptr(c, C.c_double), _ptr(a, C.c_double), a.size, s, beta, max_peaks,
                                    _ptr(Ep, C.c_double), _ptr(lp, C.c_double), C.byref(nf)))
        k = min(nf.value, max_peaks)
        return Ep[:k], lp[:k]

    def bootstrap(self, centres, a_runs, s, six_v, blo, bhi, n_boot, seed, h=1e-5, tol=1e-9):
        """beta_c and C_V peak of n_boot bootstrap samples over the runs (rows of a_runs)."""
        c, ar = _arr(centres, np.float64), _arr(np.atleast_2d(a_runs), np.float64)
        bc, pk = np.empty(n_boot), np.empty(n_boot)
        _check(lib().llr_bootstrap(self.h, _ptr(c, C.c_double), _ptr(ar, C.c_double), ar.shape[0], ar.shape[1], s,
                                   six_v, blo, bhi, h, tol, n_boot, seed, _ptr(bc, C.c_double),
                                   _ptr(pk, C.c_double)))
        return bc, pk

    # ---- observables from restricted double brackets
    def observables(self, n_meas, gap, sweep0):
        """(E, B) per measurement and interval: arrays (n_meas, total intervals)."""
        nch = sum(x[1] for x in self.lattices)
        E, B = np.empty((n_meas, nch)), np.empty((n_meas, nch))
        _check(lib().llr_observables(self.h, n_meas, gap, sweep0, _ptr(E, C.c_double), _ptr(B, C.c_double)))
        return E, B

    def obs_reconstruct(self, centres, a, s, E, B, beta):
        c, a = _arr(centres, np.float64), _arr(a, np.float64)
        E, B = _arr(np.atleast_2d(E), np.float64), _arr(np.atleast_2d(B), np.float64)
        b = _arr(np.atleast_1d(beta), np.float64)
        out = np.empty(b.size)
        _check(lib().llr_obs_reconstruct(self.h, _ptr(c, C.c_double), _ptr(a, C.c_double), a.size, s,
                                         _ptr(E, C.c_double), _ptr(B, C.c_double), E.shape[0], _ptr(b, C.c_double),
                                         b.size, _ptr(out, C.c_double)))
        return out

    # ---- multicanonical sampling and reweighting
    def muca_begin(self, b):
        """Weights W = 1/rho~ from the current a_k; b: proposal coupling per lattice."""
        b = _arr(np.broadcast_to(np.asarray(b, dtype=np.float64), (len(self.lattices),)), np.float64)
        _check(lib().llr_muca_begin(self.h, _ptr(b, C.c_double)))

    def muca_sweeps(self, n_sweeps, sweep0=0, want_E=True):
        """n_sweeps multicanonical sweeps; returns E after every sweep (n_sweeps, chains)."""
        nch = sum(x[1] for x in self.lattices)
        E = np.empty((n_sweeps, nch)) if want_E else None
        _check(lib().llr_muca_sweeps(self.h, n_sweeps, sweep0, _ptr(E, C.c_double)))
        return E

    def muca_reweight(self, E, centres, a, s, six_v, beta):
        E, c, a = _arr(np.ravel(E), np.float64), _arr(centres, np.float64), _arr(a, np.float64)
        b = _arr(np.atleast_1d(beta), np.float64)
        u, cv = np.empty(b.size), np.empty(b.size)
        _check(lib().llr_muca_reweight(self.h, _ptr(E, C.c_double), E.size, _ptr(c, C.c_double),
                                       _ptr(a, C.c_double), a.size, s, six_v, _ptr(b, C.c_double), b.size,
                                       _ptr(u, C.c_double), _ptr(cv, C.c_double)))
        return u, cv

    # ---- network
    def mlp_init(self, seed):
        w = np.empty(N_PARAMS, dtype=np.float32)
        _check(lib().llr_mlp_init(self.h, seed, _ptr(w, C.c_float)))
        return w

    def mlp_predict(self, w, u, invL, bf16=True):
        w, u, invL = _arr(w, np.float32), _arr(u, np.float32), _arr(invL, np.float32)
        a = np.empty(u.size)
        _check(lib().llr_mlp_predict(self.h, _ptr(w, C.c_float), _ptr(u, C.c_float), _ptr(invL, C.c_float), u.size,
                                     int(bf16), _ptr(a, C.c_double)))
        return a

    def mlp_warm_start(self, lattice_id, w, a_min, a_max, bf16=True):
        """Set lattice_id's a_k^(0) from the network, with the cold start
        a^(0) = 1 wherever the prediction is non-finite or outside
        [a_min, a_max].  Returns (a_k^(0), number of fallbacks)."""
        w = _arr(w, np.float32)
        n = self.lattices[lattice_id][1]
        a = np.empty(n)
        nf = C.c_int()
        _check(lib().llr_mlp_warm_start(self.h, lattice_id, _ptr(w, C.c_float), int(bf16), a_min, a_max,
                                        _ptr(a, C.c_double), C.byref(nf)))
        return a, nf.value

    def mlp_loss_grad(self, w, u, invL, a, bf16=False):
        w, u, invL, a = _arr(w, np.float32), _arr(u, np.float32), _arr(invL, np.float32), _arr(a, np.float64)
        g = np.empty(N_PARAMS, dtype=np.float32)
        loss = C.c_double()
        _check(lib().llr_mlp_loss_grad(self.h, _ptr(w, C.c_float), _ptr(u, C.c_float), _ptr(invL, C.c_float),
                                       _ptr(a, C.c_double), u.size, int(bf16), _ptr(g, C.c_float), C.byref(loss)))
        return loss.value, g

    def mlp_train(self, w, u, invL, a, epochs, lr, bf16=True):
        w = _arr(w, np.float32).copy()
        u, invL, a = _arr(u, np.float32), _arr(invL, np.float32), _arr(a, np.float64)
        hist = np.empty(max(epochs, 1))
        _check(lib().llr_mlp_train(self.h, _ptr(w, C.c_float), _ptr(u, C.c_float), _ptr(invL, C.c_float),
                                   _ptr(a, C.c_double), u.size, epochs, lr, int(bf16), _ptr(hist, C.c_double)))
        return w, hist[:epochs]


def checkpoint_info(path):
    """Validate a checkpoint on the host (no device needed) and return its
    precision, lattices [(L, E_low, dE)] and parameters."""
    prec, nl = C.c_int(), C.c_int()
    Ls = np.zeros(8, dtype=np.int32)
    ns = np.zeros(8, dtype=np.int32)
    dEs = np.zeros(8)
    prm = Params()
    _check(lib().llr_checkpoint_info(os.fsencode(path), C.byref(prec), C.byref(nl), _ptr(Ls, C.c_int),
                                     _ptr(ns, C.c_int), _ptr(dEs, C.c_double), None, C.byref(prm)))
    E_low = np.zeros(int(ns[: nl.value].sum()))
    _check(lib().llr_checkpoint_info(os.fsencode(path), None, None, None, None, None, _ptr(E_low, C.c_double), None))
    lats, off = [], 0
    for i in range(nl.value):
        lats.append((int(Ls[i]), E_low[off: off + ns[i]].copy(), float(dEs[i])))
        off += int(ns[i])
    return {"precision": prec.value, "lattices": lats, "params": prm}


def fss_fit(L, y, sigma, powers):
    """Weighted least squares y(L) = sum_j p_j L^powers_j: (params, errors, chi2_red)."""
    L, y, sg, pw = (_arr(v, np.float64) for v in (L, y, sigma, powers))
    p, e, chi2 = np.empty(pw.size), np.empty(pw.size), C.c_double()
    _check(lib().llr_fss_fit(_ptr(L, C.c_double), _ptr(y, C.c_double), _ptr(sg, C.c_double), L.size,
                             _ptr(pw, C.c_double), pw.size, _ptr(p, C.c_double), _ptr(e, C.c_double),
                             C.byref(chi2)))
    return p, e, chi2.value
