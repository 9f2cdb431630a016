"""Pins of the oracle's fiber migration (Sec. 3.5.2): the paper switches
periodically and randomly between fiber tables of distinct fiber
arrangements and interpolates between them.  The reading: table 0 is the
regular arrangement, table m > 0 pulls every fiber inwards by a drawn
factor, each period of the ply's arc length picks a table per ply, and the
last share of a period blends linearly into the next period's table.

Checked against computations that do not go through the oracle's code:
Philox4x32-10 written here from its published definition (pinned by the
known-answer file), perturbed fiber arrangements cast by dense marching,
and the reading's own limits (no spread reduces to the regular model; the
values are continuous along the ply; outside the blend they are one
table's)."""
import math

import numpy as np
import pytest

from paper_2401_12724_amd import workloads as W

from test_oracle_bruteforce import _blocked_fraction, _first_inside, _vogel

M32 = 0xFFFFFFFF


def _philox(ctr, key):
    """Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32
    multiplications, the Weyl key schedule between rounds."""
    c = [x & M32 for x in ctr]
    k0, k1 = key[0] & M32, key[1] & M32
    for r in range(10):
        p0 = 0xD2511F53 * c[0]
        p1 = 0xCD9E8D57 * c[2]
        hi0, lo0 = p0 >> 32, p0 & M32
        hi1, lo1 = p1 >> 32, p1 & M32
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
        if r < 9:
            k0 = (k0 + 0x9E3779B9) & M32
            k1 = (k1 + 0xBB67AE85) & M32
    return c


def test_python_philox_matches_known_answers():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")
    n = 0
    for line in open(path):
        line = line.split("#")[0].split()
        if len(line) != 10:
            continue
        v = [int(x, 16) for x in line]
        assert _philox(v[0:4], v[4:6]) == v[6:10]
        n += 1
    assert n >= 3


def _params(**kw):
    return W.default_params(**dict(dict(mig_tables=4, mig_period=3.0, mig_blend=0.25,
                                        mig_spread=0.4, mig_seed=11), **kw))


def test_no_spread_reduces_to_the_regular_model(oracle_mod):
    """With no spread every table is the regular one, so evaluation and
    sampling equal the model without migration (up to the rounding of the
    blend (1 - w) a + w a)."""
    P0 = W.default_params()
    P1 = _params(mig_spread=0.0)
    _, q = W.single_type(4000, 21, with_xi=True)
    a, af = oracle_mod.eval([P0], q)
    b, bf = oracle_mod.eval([P1], q)
    assert np.array_equal(af, bf)
    assert np.allclose(a, b, rtol=1e-9, atol=1e-12)
    sa, _ = oracle_mod.sample([P0], q)
    sb, _ = oracle_mod.sample([P1], q)
    assert np.allclose(sa, sb, rtol=1e-9, atol=1e-12)


def test_migration_changes_the_model(oracle_mod):
    """With spread the switching tables change the values along the ply."""
    _, q = W.single_type(4000, 22)
    a, _ = oracle_mod.eval([W.default_params()], q)
    b, _ = oracle_mod.eval([_params()], q)
    assert np.mean(np.abs(a - b).max(1) > 1e-6) > 0.2


def test_table_choice_is_the_drawn_one(oracle_mod):
    P = _params()
    for q in (-3, 0, 1, 7, 2 ** 33 + 5):
        for k in range(3):
            uq = q & 0xFFFFFFFFFFFFFFFF
            w = _philox([uq & M32, uq >> 32, k, 0x53454C54], [P["mig_seed"], 0x46494252])
            assert oracle_mod.mig_table(P, q, k) == w[0] % 4


@pytest.mark.parametrize("m", [1, 3])
def test_perturbed_table_bruteforce(oracle_mod, m):
    """Table m against dense casting through the perturbed arrangement,
    built here from the Philox draws."""
    M, rho, Nu = 32, 0.08, 256
    P = _params(fibers_per_ply=M, fiber_radius=rho, tex_size=Nu)
    tab = oracle_mod.table(P)[m * Nu:(m + 1) * Nu]
    C = _vogel(M, rho)
    for j in range(M):
        w = _philox([j, m, 0x4D494752, 0], [P["mig_seed"], 0x46494252])
        f = min(1.0, 1.0 + P["mig_spread"] * (2.0 * (w[0] >> 8) / 2.0 ** 24 - 1.0))
        C[j] *= f
    rng = np.random.default_rng(m)
    for i in rng.choice(Nu, 20, replace=False):
        z = 2 * math.pi * (i + 0.5) / Nu
        e = np.array([math.cos(z), math.sin(z)])
        s, j = _first_inside(1.0000001 * e, -e, C, rho, 2.0, rho / 50)
        if j < 0:
            assert tab[i, 1] == 0.0 and tab[i, 2] == 1.0 and tab[i, 0] == 0.0
            continue
        qp = 1.0000001 * e - s * e
        n = (qp - C[j]) / rho
        assert abs(tab[i, 0] - math.atan2(e[0] * n[1] - e[1] * n[0], e @ n)) < 1e-5
        assert abs(tab[i, 1] - np.linalg.norm(C[j]) / (1 - rho)) < 1.2e-7
        assert abs(tab[i, 2] - (1.0 - _blocked_fraction(qp, n, np.delete(C, j, 0), rho))) < 2e-3


def test_lookup_is_one_table_outside_the_blend(oracle_mod):
    P = _params()
    tab = oracle_mod.table(P)
    Nu, L = P["tex_size"], P["mig_period"]
    single = dict(P, mig_tables=1)
    rng = np.random.default_rng(3)
    for _ in range(50):
        qd, k = int(rng.integers(-5, 40)), int(rng.integers(0, 3))
        ph = rng.uniform(0.0, 0.74)
        uf = rng.uniform(-20, 20)
        v = (qd + ph) * L
        m = oracle_mod.mig_table(P, qd, k)
        want = oracle_mod.fiber_lookup(single, tab[m * Nu:(m + 1) * Nu], uf, v, k)
        got = oracle_mod.fiber_lookup(P, tab, uf, v, k)
        assert np.allclose(got, want, rtol=0, atol=1e-12)


def test_lookup_blends_linearly_and_is_continuous(oracle_mod):
    P = _params()
    tab = oracle_mod.table(P)
    Nu, L, b = P["tex_size"], P["mig_period"], P["mig_blend"]
    single = dict(P, mig_tables=1)
    rng = np.random.default_rng(4)
    for _ in range(50):
        qd, k = int(rng.integers(-5, 40)), int(rng.integers(0, 3))
        uf = rng.uniform(-20, 20)
        ph = rng.uniform(1 - b, 1.0)
        v = (qd + ph) * L
        w = (v / L - math.floor(v / L) - (1 - b)) / b
        m0, m1 = oracle_mod.mig_table(P, qd, k), oracle_mod.mig_table(P, qd + 1, k)
        a = oracle_mod.fiber_lookup(single, tab[m0 * Nu:(m0 + 1) * Nu], uf, v, k)
        c = oracle_mod.fiber_lookup(single, tab[m1 * Nu:(m1 + 1) * Nu], uf, v, k)
        assert np.allclose(oracle_mod.fiber_lookup(P, tab, uf, v, k), (1 - w) * a + w * c,
                           rtol=0, atol=1e-12)
        # continuity at the period boundary and where the blend starts
        for vb in ((qd + 1) * L, (qd + 1 - b) * L):
            lo = oracle_mod.fiber_lookup(P, tab, uf, vb - 1e-9, k)
            hi = oracle_mod.fiber_lookup(P, tab, uf, vb + 1e-9, k)
            assert np.abs(lo - hi).max() < 1e-6
