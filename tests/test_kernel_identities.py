"""Arithmetic identities the HIP kernels rely on, checked on the CPU in the
kernels' own IEEE formats (numpy binary64 / binary32, round to nearest even).
They do not call the kernels; the GPU parity tests check the kernels.

* fixed-point rounding without a float-to-integer conversion: adding
  1.5 * 2^52 to v * 2^32 (|v| < 2^18) leaves rint(v * 2^32) in the low bits
  of the sum's significand;
* the bin of a fixed-point energy from a binary64 quotient estimate (E - e_min
  times 1 / bin_w) corrected by one exact integer step equals the floor
  division, clamped to +-2^30;
* the closed form of n sequential additions of ln f to one ln g value (the
  speculative commit): after the first add every add moves the value by the
  same exact step while it stays in one binade, in binary64, and for the
  (hi, lo) pair whose high word ln f leaves unchanged, in the low word.
"""
import numpy as np

F64, F32 = np.float64, np.float32


def fx_magic(v):
    y = v * 2.0**32 + 1.5 * 2.0**52
    return y.view(np.int64) - 0x4338000000000000


def test_fixed_point_rounding_without_conversion():
    rng = np.random.default_rng(11)
    v = np.concatenate([rng.uniform(-2**18, 2**18, 200_000), rng.normal(0.0, 1.0, 200_000),
                        (rng.integers(-2**40, 2**40, 50_000) + 0.5) / 2**32,      # exact ties
                        np.array([0.0, -0.0, 2**18 - 2**-30, -(2**18 - 2**-30), 1e-300, 2**-33, 3 * 2**-33])])
    v = v[np.abs(v) < 2**18]
    assert np.array_equal(fx_magic(v), np.rint(v * 2.0**32).astype(np.int64))


def fx_bin_estimate(diff, bw):
    inv = 1.0 / float(bw)
    qd = np.floor(float(diff) * inv)
    if qd <= -1073741825.0:
        return -2**30
    if qd >= 1073741825.0:
        return 2**30
    q = int(qd)
    if q * bw > diff:
        q -= 1
    elif (q + 1) * bw <= diff:
        q += 1
    return max(-2**30, min(2**30, q))


def test_bin_from_corrected_binary64_quotient():
    rng = np.random.default_rng(12)
    widths = [1, 3, 2**31, 2**31 + 1, 2**32, 10**9 + 7, 2**60]
    for _ in range(40_000):
        bw = int(rng.choice(widths)) if rng.random() < 0.5 else int(rng.integers(1, 2**60))
        if rng.random() < 0.6:
            q = int(rng.integers(-2**31, 2**31))
            diff = q * bw + int(rng.choice([0, 1, -1, bw - 1, int(rng.integers(0, bw))]))
        else:
            diff = int(rng.integers(-2**62 + 1, 2**62))
        if abs(diff) >= 2**62:
            continue
        assert fx_bin_estimate(diff, bw) == max(-2**30, min(2**30, diff // bw)), (diff, bw)


def closed_form_f64(c, x, n):
    """(applies, value) of n sequential adds of x to c by the kernel's closed form."""
    x1 = F64(c + x)
    d2 = F64(F64(x1 + x) - x1)
    _, ex = np.frexp(x1)
    top = np.ldexp(F64(1.0), int(ex))
    nm1 = F64(n - 1)
    if d2 * 64.0 <= x1 and x1 + nm1 * d2 + 4.0 * x < top * (1.0 - 2.0**-40):
        return True, F64(x1 + F64(nm1 * d2))
    return False, None


def test_binary64_replay_closed_form_equals_sequential_adds():
    rng = np.random.default_rng(13)
    used = 0
    for _ in range(60_000):
        c = F64(rng.choice([0.5, 7.0, 300.0, 2500.0, 1.5e5]) * rng.uniform(0.5, 2.0))
        x = F64(rng.choice([3.6e-7, 1e-8, 2.0**-20, 1.0 / (3 * 2**17), 2.0**-9, 1e-3]))
        n = int(rng.integers(1, 65))
        ok, val = closed_form_f64(c, x, n)
        if not ok:
            continue
        used += 1
        ref = c
        for _ in range(n):
            ref = F64(ref + x)
        assert val == ref, (c, x, n)
    assert used > 30_000


def two_sum_add(h, l, x):
    s = F32(h + x)
    bb = F32(s - h)
    err = F32(F32(h - F32(s - bb)) + F32(x - bb))
    return s, F32(l + err)


def test_pair_low_word_replay_closed_form_equals_sequential_two_sums():
    rng = np.random.default_rng(14)
    used = 0
    for _ in range(60_000):
        h = F32(rng.choice([1.0, 40.0, 300.0, 2000.0, -1700.0, 5e4]) * rng.uniform(0.5, 1.5))
        x = F32(rng.choice([3.6e-7, 1e-6, 2.0**-20, 2.0**-12, 1e-8, 3e-6]))
        l = F32(rng.choice([0.0, 1.0, -1.0]) * rng.uniform(0.0, 1.0) * float(np.spacing(h))
                * rng.choice([0.1, 0.5, 3.0, 100.0]))
        n = int(rng.integers(1, 65))
        if F32(h + x) != h:
            continue                        # the kernel takes the add-by-add path
        x1 = F32(l + x)
        d2 = F32(F32(x1 + x) - x1)
        _, ex = np.frexp(x1)
        top = np.ldexp(F32(1.0), int(ex))
        nm1 = F32(n - 1)
        if not (F32(d2 * F32(64.0)) <= x1 and
                float(x1) + float(nm1) * float(d2) + 4.0 * float(x) < float(top) * (1.0 - 2.0**-20)):
            continue
        used += 1
        hh, ll = h, l
        for _ in range(n):
            hh, ll = two_sum_add(hh, ll, x)
        assert hh == h and F32(x1 + F32(nm1 * d2)) == ll, (h, l, x, n)
    assert used > 5_000
