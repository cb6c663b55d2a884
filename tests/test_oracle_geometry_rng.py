"""Oracle pins: lattice geometry and colouring by brute force (Sec. 3.1 plaquette
definition), Philox4x32-10 against published known answers and against the
independent implementation in PyTorch's ATen headers, uniform conversions, and
the von Mises heatbath sampler against scipy's distribution and Bessel-ratio
moments (Best & Fisher 1979)."""
import itertools
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest
from scipy import special, stats

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _coords(s, d, L):
    return tuple((s // L ** m) % L for m in range(d))


def _site(x, L):
    return sum(c * L ** m for m, c in enumerate(x))


@pytest.mark.parametrize("d,L", [(2, 2), (2, 4), (2, 6), (4, 2), (4, 4)])
def test_neighbours_and_colouring_brute_force(d, L):
    V = L ** d
    for s in range(V):
        x = _coords(s, d, L)
        for mu in range(d):
            for step in (+1, -1):
                y = list(x)
                y[mu] = (y[mu] + step) % L
                assert oracle.neighbour(d, L, s, mu, step) == _site(y, L)
    # enumerate plaquettes (x, mu < nu): links (mu,x), (nu,x+mu), (mu,x+nu), (nu,x)
    count = {}
    for s in range(V):
        x = _coords(s, d, L)
        for mu, nu in itertools.combinations(range(d), 2):
            xm = list(x); xm[mu] = (xm[mu] + 1) % L
            xn = list(x); xn[nu] = (xn[nu] + 1) % L
            links = [(mu, s), (nu, _site(xm, L)), (mu, _site(xn, L)), (nu, s)]
            colours = []
            for (m, t) in links:
                p = sum(_coords(t, d, L)) % 2
                colours.append(2 * m + p)
                count[(m, t)] = count.get((m, t), 0) + 1
            # no two links of one plaquette share a colour (for L >= 4; at L = 2
            # the periodic wrap makes x+nu and x-nu coincide, which is still a
            # different parity)
            assert len(set(colours)) == 4
    assert len(count) == d * V
    assert set(count.values()) == {2 * (d - 1)}
    assert sum(count.values()) == 4 * V * d * (d - 1) // 2


def _load_kat():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            rows.append([int(t, 16) for t in line.split()])
    return rows


def test_philox_known_answers():
    for r in _load_kat():
        ctr = np.array([r[0:4]], dtype=np.uint32)
        seed = r[4] | (r[5] << 32)
        out = oracle.philox(ctr, seed)[0]
        assert [int(v) for v in out] == r[6:10]


TORCH_KAT = r'''
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
#include <cstdlib>
int main(int argc, char** argv) {
  unsigned long long seed = strtoull(argv[1], 0, 10);
  for (int i = 0; i < 2000; ++i) {
    unsigned c0 = 977u * i + 3u, c1 = 0x00012300u + i, c2 = 5u * i, c3 = 11u * i + 1u;
    unsigned long long sub = ((unsigned long long)c3 << 32) | c2;
    unsigned long long off = ((unsigned long long)c1 << 32) | c0;
    at::Philox4_32 e(seed, sub, off);
    unsigned a = e(), b = e(), c = e(), d = e();
    printf("%u %u %u %u %u %u %u %u\n", c0, c1, c2, c3, a, b, c, d);
  }
  return 0;
}
'''


def test_philox_against_aten_engine(tmp_path):
    """Cross-check with the independent Philox4x32-10 of PyTorch's ATen header
    (compiled and called here, nothing copied)."""
    import torch
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    if not os.path.exists(os.path.join(inc, "ATen", "core", "PhiloxRNGEngine.h")) or not shutil.which("g++"):
        pytest.skip("ATen header or g++ not available")
    src = tmp_path / "kat.cpp"
    src.write_text(TORCH_KAT)
    exe = tmp_path / "kat"
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-I", inc, str(src), "-o", str(exe)])
    seed = 1509083910 | (77 << 32)
    out = subprocess.check_output([str(exe), str(seed)]).decode().split("\n")
    rows = np.array([[int(t) for t in l.split()] for l in out if l.strip()], dtype=np.uint64)
    mine = oracle.philox(rows[:, :4].astype(np.uint32), seed)
    assert np.array_equal(mine.astype(np.uint64), rows[:, 4:])


def test_uniform_conversions_exact_and_open():
    w = np.array([0, 1, 255, 256, 2 ** 31 - 1, 2 ** 31, 2 ** 32 - 1], dtype=np.uint32)
    u, v = oracle.uniforms(w, u24=False)
    assert np.all(u > 0) and np.all(u < 1) and np.all(np.abs(v) < 1)
    assert u[0] == 0.5 * 2.0 ** -32 and u[-1] == 1 - 0.5 * 2.0 ** -32
    assert v[5] == -1 + 0.5 * 2.0 ** -31 and v[4] == 1 - 0.5 * 2.0 ** -31
    u, v = oracle.uniforms(w, u24=True)
    assert np.all(u > 0) and np.all(u < 1) and np.all(np.abs(v) < 1)
    assert np.all(u.astype(np.float32).astype(np.float64) == u)
    assert np.all(v.astype(np.float32).astype(np.float64) == v)
    # the signed uniform is symmetric: w and ~w map to -v
    _, v1 = oracle.uniforms(w, u24=False)
    _, v2 = oracle.uniforms(~w, u24=False)
    assert np.array_equal(v1, -v2)
    # chi-square uniformity of Philox output over 64 bins
    ctr = np.zeros((200000, 4), dtype=np.uint32)
    ctr[:, 0] = np.arange(200000)
    u, _ = oracle.uniforms(oracle.philox(ctr, 99).ravel())
    h, _ = np.histogram(u, bins=64, range=(0, 1))
    assert stats.chisquare(h).pvalue > 1e-4


@pytest.mark.parametrize("kappa", [0.0, 1e-6, 0.5, 2.0, 6.0, 12.0])
@pytest.mark.parametrize("u24", [False, True])
def test_vonmises_sampler_distribution(kappa, u24):
    n = 400000
    X, att, _ = oracle.vonmises(n, kappa, seed=2024 + int(10 * kappa), c1=oracle.ctr1(kind=0), u24=u24)
    assert np.all(att > 0) and np.all(np.abs(X) <= np.pi)
    if kappa > 0:
        cdf = stats.vonmises(kappa).cdf
    else:
        cdf = stats.uniform(-np.pi, 2 * np.pi).cdf
    assert stats.kstest(X, cdf).pvalue > 1e-3
    for m in (1, 2):
        exp = special.ive(m, kappa) / special.ive(0, kappa) if kappa > 0 else 0.0
        got = np.mean(np.cos(m * X))
        sd = np.std(np.cos(m * X)) / np.sqrt(n)
        assert abs(got - exp) < 5 * sd + 1e-12
    assert abs(np.mean(np.sin(X))) < 5 / np.sqrt(n)
    # Best-Fisher efficiency bound: mean attempts below 1/0.65
    assert att.mean() < 1.0 / 0.65
