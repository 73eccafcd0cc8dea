"""Pins for the oracle's scalar building blocks, each against something other
than the oracle itself: numpy's Philox, libm's exp in FP64, closed forms of
the Intelligent Driver Model (Eq. (1)), binomial frequencies of Eq. (2),
hand-computed cases of Eqs. (3)-(4)."""
import math

import numpy as np
import pytest

SEED = 1234


def numpy_philox_block(counter, key):
    """numpy's Philox4x64-10 increments its 256-bit counter before each block,
    so the block at counter c is the first output of a generator started at c-1."""
    c = [int(x) for x in counter]
    # subtract one with borrow across the four 64-bit words
    for q in range(4):
        if c[q] > 0:
            c[q] -= 1
            break
        c[q] = (1 << 64) - 1
    bg = np.random.Philox(counter=np.array(c, dtype=np.uint64), key=np.array(key, dtype=np.uint64))
    return bg.random_raw(4)


@pytest.mark.parametrize("counter,key", [
    ([1, 0, 0, 0], [5, 0]),
    ([0, 0, 0, 0], [0, 0]),
    ([7, 123456, 2, 1], [SEED, 0]),
    ([2**63 + 5, 2**40, 3, 2], [2**64 - 1, 0]),
    ([123, 0, 0, 0], [987654321, 0]),
])
def test_philox_matches_numpy(oracle_mod, counter, key):
    ours = oracle_mod.philox4x64(counter, key)
    ref = numpy_philox_block(counter, key)
    assert ours.tolist() == ref.tolist()


def test_uniform_and_normal_from_numpy_words(oracle_mod):
    rng = np.random.default_rng(0)
    for _ in range(50):
        t = int(rng.integers(0, 50_000))
        vid = int(rng.integers(0, 3_000_000))
        w0 = numpy_philox_block([t, vid, 1, 0], [SEED, 0])
        u = np.float32(int(w0[0]) >> 40) * np.float32(2.0 ** -24)
        assert oracle_mod.uniform(SEED, t, vid, 1) == float(u)
        words = np.concatenate([numpy_philox_block([t, vid, 2, b], [SEED, 0]) for b in range(3)])
        S = sum(int(x) >> 40 for x in words)
        eps = np.float32(np.int32(S - 6 * 2**24)) * np.float32(2.0 ** -24)
        assert oracle_mod.normal(SEED, t, vid, 2) == float(eps)
        # the FP64 twin uses the same integers, without the FP32 rounding
        assert oracle_mod.normal(SEED, t, vid, 2, fp64=True) == (S - 6 * 2**24) * 2.0 ** -24


def test_irwin_hall_moments(oracle_mod):
    """Irwin-Hall(12) - 6 on 24-bit grids: mean -12 * 2^-25, variance 1 - 2^-48
    (each 24-bit uniform has variance (1 - 2^-48)/12); tails cut at +-6."""
    n = 40_000
    x = np.array([oracle_mod.normal(SEED, 17, i, 3, fp64=True) for i in range(n)])
    assert abs(x.mean() - (-12 * 2.0 ** -25)) < 5.0 / math.sqrt(n)
    assert abs(x.var() - 1.0) < 6.0 * math.sqrt(2.0 / n)
    assert np.abs(x).max() < 6.0
    # fourth central moment of Irwin-Hall(12) - 6 is 3 - 1.2/12 = 2.9
    m4 = ((x - x.mean()) ** 4).mean()
    assert abs(m4 - 2.9) < 0.15


def test_expf_c_within_2ulp(oracle_mod):
    """exp(y) on (-17, 0] against FP64 libm: a dense sample of FP32 inputs."""
    bits_lo = np.float32(-17.0).view(np.uint32)       # negative floats: larger bits = more negative
    ys = np.arange(0x80000000, int(bits_lo), 97, dtype=np.uint64).astype(np.uint32).view(np.float32)
    ys = np.concatenate([ys, np.array([0.0, -0.0, -1e-30, -0.34657359, -0.6931472, -16.999998,
                                       -np.float32(1e-7)], np.float32)])
    ours = oracle_mod.expf_c(ys)
    ref = np.exp(ys.astype(np.float64))
    ulp = np.spacing(ref.astype(np.float32)).astype(np.float64)
    err = np.abs(ours.astype(np.float64) - ref) / ulp
    assert err.max() <= 2.0, (err.max(), ys[np.argmax(err)])
    assert oracle_mod.expf_c(np.array([0.0], np.float32))[0] == 1.0


# ---------------------------------------------------------------- Eq. (1)
V0 = np.float32(50.0 / 3.6)


def s_equilibrium(v, v0=float(V0), s0=2.0, T=1.5):
    """Platoon equilibrium gap of the IDM with delta = 4 (Delta v = 0)."""
    return (s0 + v * T) / math.sqrt(1.0 - (v / v0) ** 4)


@pytest.mark.parametrize("v", [5.0, 10.0, 12.0, 13.0])
def test_idm_platoon_equilibrium(oracle_mod, v):
    s = s_equilibrium(v)
    acc32, fl = oracle_mod.idm(v, float(V0), v, s, 1.5, 1.0, 2.0, 2.0, kind=1)
    assert fl == 0
    assert abs(acc32) < 2e-5          # FP32 rounding of O(1) terms
    acc64, _ = oracle_mod.idm(v, float(V0), v, s, 1.5, 1.0, 2.0, 2.0, kind=1, fp64=True)
    assert abs(acc64) < 1e-12


def test_idm_fixed_points(oracle_mod):
    # standstill queue at the jam gap: exactly zero
    acc, fl = oracle_mod.idm(0.0, float(V0), 0.0, 2.0, 1.5, 1.0, 2.0, 2.0, kind=1)
    assert acc == 0.0 and fl == 0
    # free road at the desired speed: exactly zero
    acc, _ = oracle_mod.idm(float(V0), float(V0), 0.0, 0.0, 1.5, 1.0, 2.0, 2.0, kind=0)
    assert acc == 0.0
    # free road from rest: exactly a
    acc, _ = oracle_mod.idm(0.0, float(V0), 0.0, 0.0, 1.5, 1.7, 2.0, 2.0, kind=0)
    assert acc == np.float32(1.7)


def test_idm_branches(oracle_mod):
    # A3: far above v0 the free term is floored at -b
    acc, fl = oracle_mod.idm(30.0, 10.0, 0.0, 0.0, 1.5, 1.0, 2.0, 2.0, kind=0)
    assert fl & 1 and acc == -2.0
    # A1: a much faster leader makes the dynamic term negative -> s* = s0
    acc, fl = oracle_mod.idm(5.0, float(V0), 20.0, 10.0, 1.5, 1.0, 2.0, 2.0, kind=1)
    assert fl & 2
    r = 5.0 / float(V0)
    assert acc == pytest.approx(1.0 * (1 - r ** 4) - 1.0 * (2.0 / 10.0) ** 2, rel=1e-6)
    # A4: the gap is floored at 0.1 m
    acc, fl = oracle_mod.idm(0.0, float(V0), 0.0, 0.0, 1.5, 1.0, 2.0, 2.0, kind=1)
    assert fl & 4 and acc == pytest.approx(1.0 - (2.0 / 0.1) ** 2, rel=1e-6)


# ---------------------------------------------------------------- Eq. (2)
def test_mandatory_certain_within_x0(oracle_mod):
    for vid in range(200):
        for d in (0.0, 0.5, 1.0):
            assert oracle_mod.mand_trigger(SEED, 3, vid, d) == 1


@pytest.mark.parametrize("d", [1.5, 2.0, 2.5, 3.0])
def test_mandatory_frequency(oracle_mod, d):
    n = 20_000
    hits = sum(oracle_mod.mand_trigger(SEED, 11, vid, d) for vid in range(n))
    p = math.exp(-(d - 1.0) ** 2)
    sd = math.sqrt(p * (1 - p) / n)
    assert abs(hits / n - p) < 4.5 * sd + 1e-4


def test_mandatory_never_far(oracle_mod):
    assert sum(oracle_mod.mand_trigger(SEED, 5, vid, 6.0) for vid in range(5000)) == 0


# ---------------------------------------------------------------- Eqs. (3)-(4)
def test_gap_acceptance_hand_cases(oracle_mod):
    # zero anticipation: the critical gap is the desired gap
    assert oracle_mod.crit_gap(3.0, 0.0, 10.0, 0.0, 4.0) == 3.0
    # g0 + alpha_a v_i + alpha_i (v_i - v_a) = 3 + 0.2*10 + 0.3*5 = 6.5
    assert oracle_mod.crit_gap(3.0, 0.2, 10.0, 0.3, 5.0) == pytest.approx(6.5, abs=1e-6)
    # a fast other vehicle makes the speed terms negative: floored at g0
    assert oracle_mod.crit_gap(3.0, 0.1, 1.0, 0.4, 20.0) == 3.0
    assert oracle_mod.crit_gap(7.5, 0.05, 12.0, 0.05, 12.0) == pytest.approx(8.1, abs=1e-6)
    # desired gap: 1-5 m below 25 mph (midpoint 3), 5-10 m above (midpoint 7.5)
    assert oracle_mod.desired_gap(11.0) == 3.0
    assert oracle_mod.desired_gap(11.2) == 7.5
    assert oracle_mod.desired_gap(float(np.float32(11.176))) == 7.5
