"""Pins of the Eq. 5 reading (paper Sec. 5.1, Eq. 5): the mean, over the bins
whose reference is non-zero, of |ref - y| / |ref|.

The printed formula is garbled (a lower-case x in the denominator and a sum
running to N); the reading taken here divides by the modulus of the FP64
reference bin and skips bins where that modulus is zero.  The pins below are
hand-computed values and special cases, so that a plausible slip (dividing by
|y|, counting zero-reference bins, summing instead of averaging, or squaring
the moduli) fails at least one of them; each slip is planted in a copy of the
function and must be caught."""
import math

import numpy as np
import pytest

import oracle


def pin_hand_example(f):
    """Four bins, one zero reference bin; by hand:
    bin 0: ref 2,      y 2.5      -> |0.5| / 2 = 0.25
    bin 1: ref 0,      y 7        -> skipped (reference zero)
    bin 2: ref 3+4i,   y 3+3i     -> |i| / 5   = 0.2
    bin 3: ref -1i,    y 0        -> |-1i| / 1 = 1
    mean over the three counted bins = 1.45 / 3."""
    ref = np.array([2.0, 0.0, 3 + 4j, -1j])
    y = np.array([2.5, 7.0, 3 + 3j, 0.0])
    got = f(y, ref)
    assert abs(got - 1.45 / 3) < 1e-15, got


def pin_uniform_relative_perturbation(f):
    """y = ref (1 + eps e^{i phi}) has |ref - y| / |ref| = eps in every bin."""
    g = np.random.default_rng(5)
    ref = g.standard_normal(64) + 1j * g.standard_normal(64)
    for eps in (1e-3, 0.25, 2.0):
        y = ref * (1 + eps * np.exp(1j * g.uniform(0, 2 * math.pi, 64)))
        got = f(y, ref)
        assert abs(got - eps) < 1e-12 * max(1.0, eps), (eps, got)


def pin_exact_and_zero_cases(f):
    """An exact result reads 0; an all-zero reference reads 0 (no bin counts);
    the shape of the arrays does not matter (the mean runs over all bins)."""
    g = np.random.default_rng(6)
    ref = g.standard_normal((3, 8)) + 1j * g.standard_normal((3, 8))
    assert f(ref.copy(), ref) == 0.0
    assert f(np.ones(5, complex), np.zeros(5, complex)) == 0.0
    y = ref * 1.5
    assert abs(f(y, ref) - 0.5) < 1e-14
    assert abs(f(y.ravel(), ref.ravel()) - f(y, ref)) < 1e-15


def pin_single_bad_bin(f):
    """One bin off by 100 % among 10 exact ones: the mean is 1/10 whatever
    the modulus of that bin (large or tiny), which a division by |y| or a
    squared modulus would change."""
    for mag in (1e-4, 1.0, 1e4):
        ref = np.full(10, 1 + 1j)
        ref[3] = mag * (1 - 2j)
        y = ref.copy()
        y[3] = 0.0
        got = f(y, ref)
        assert abs(got - 0.1) < 1e-14, (mag, got)


PINS = [pin_hand_example, pin_uniform_relative_perturbation, pin_exact_and_zero_cases,
        pin_single_bad_bin]


@pytest.mark.parametrize("pin", PINS, ids=lambda p: p.__name__)
def test_eq5_pin(pin):
    pin(oracle.eq5_error)


# Plausible slips planted in copies of the reading (never in the oracle).
def _divide_by_y(y, ref):
    y, ref = np.ravel(y), np.ravel(ref)
    m = np.abs(y) > 0
    return float(np.mean(np.abs(ref[m] - y[m]) / np.abs(y[m]))) if m.any() else 0.0


def _zero_bins_counted(y, ref):
    y, ref = np.ravel(y), np.ravel(ref)
    m = np.abs(ref) > 0
    num = np.where(m, np.abs(ref - y) / np.where(m, np.abs(ref), 1.0), 0.0)
    return float(np.mean(num))


def _sum_not_mean(y, ref):
    y, ref = np.ravel(y), np.ravel(ref)
    m = np.abs(ref) > 0
    return float(np.sum(np.abs(ref[m] - y[m]) / np.abs(ref[m])))


def _squared(y, ref):
    y, ref = np.ravel(y), np.ravel(ref)
    m = np.abs(ref) > 0
    return float(np.mean(np.abs(ref[m] - y[m]) ** 2 / np.abs(ref[m]) ** 2)) if m.any() else 0.0


def _real_parts_only(y, ref):
    y, ref = np.ravel(y), np.ravel(ref)
    m = np.abs(ref) > 0
    return float(np.mean(np.abs(ref[m].real - y[m].real) / np.abs(ref[m]))) if m.any() else 0.0


MUTANTS = [_divide_by_y, _zero_bins_counted, _sum_not_mean, _squared, _real_parts_only]


@pytest.mark.parametrize("mutant", MUTANTS, ids=lambda m: m.__name__)
def test_eq5_mutant_is_caught(mutant):
    caught = []
    for pin in PINS:
        try:
            pin(mutant)
        except AssertionError:
            caught.append(pin.__name__)
    assert caught, f"{mutant.__name__} passed every Eq. 5 pin"
