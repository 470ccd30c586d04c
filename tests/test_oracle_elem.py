"""Pins for the oracle's own exp, expm1, log and log1p (used by the heat-bath draw and
the Gaussian couplings) and for the heat-bath bookkeeping.

The constants are compared with exact rational values rounded once (1/n!, 1/(2j+1),
ln 2 from a 60-digit decimal evaluation); the functions with high-precision
references (binary64 library values for binary32, 60-digit decimal arithmetic for
binary64); the device's literal constants, read from its header as text, with the
same exact values.
"""
from __future__ import annotations

import math
import os
import re
from decimal import Decimal, getcontext
from fractions import Fraction as F

import numpy as np
import pytest

import oracle as O

F32, F64 = np.float32, np.float64
MANT = {F32: 24, F64: 53}
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
getcontext().prec = 60
LN2 = F(Decimal(2).ln())
SQRT_HALF = F(Decimal("0.5").sqrt())


def round_to(fr: F, bits: int) -> F:
    """Exact rational rounded to a binary significand of `bits` bits, ties to even."""
    if fr == 0:
        return F(0)
    sign, a = (-1 if fr < 0 else 1), abs(fr)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    while F(2) ** e > a:
        e -= 1
    while F(2) ** (e + 1) <= a:
        e += 1
    x = a * F(2) ** (bits - 1 - e)
    n, rem = divmod(x.numerator, x.denominator)
    rem = F(rem, x.denominator)
    if rem > F(1, 2) or (rem == F(1, 2) and n % 2):
        n += 1
    return sign * F(n) / F(2) ** (bits - 1 - e)


def expected_consts(dtype):
    bits = MANT[dtype]
    expm1 = [round_to(F(1, math.factorial(n)), bits) for n in range(18)]
    atanh = [round_to(F(1, 2 * j + 1), bits) for j in range(18)]
    split = 16 if dtype == F32 else 32
    head = F(round(LN2 * 2 ** split), 2 ** split)
    ln2 = [head, round_to(LN2 - head, bits), round_to(1 / LN2, bits), round_to(SQRT_HALF, bits)]
    return expm1, atanh, ln2


@pytest.mark.parametrize("dtype", [F32, F64])
def test_constants_are_correctly_rounded(dtype):
    got = O.elem_consts(dtype)
    for g, want in zip(got, expected_consts(dtype)):
        assert [F(float(v)) for v in g] == want
    head = F(float(got[2][0]))
    # the head times any exponent of the format is exact
    split_bits = (head * 2 ** (16 if dtype == F32 else 32)).denominator
    assert split_bits == 1


def test_device_literals_are_correctly_rounded():
    """The device header spells the same constants as literals: each equals the
    correctly rounded exact value."""
    text = open(os.path.join(ROOT, "paper_1006_2566_amd", "csrc", "hsg_device.h")).read()
    for dtype, tag in ((F32, "Elem<float>"), (F64, "Elem<double>")):
        body = text[text.index(f"struct {tag} {{"):]
        body = body[:body.index("\n};")]
        expm1, atanh, ln2 = expected_consts(dtype)
        lit = {m.group(2): F(float.fromhex(m.group(1).rstrip("f")))
               for m in re.finditer(r"(-?0x[0-9a-fp.+-]+f?)\)?;\s*// 1/(\d+!?)", body)}
        for n in range(2, 9 if dtype == F32 else 14):
            assert lit[f"{n}!"] == expm1[n], (tag, n)
        for j in range(1, 8 if dtype == F32 else 18):
            assert lit[str(2 * j + 1)] == atanh[j], (tag, j)
        # the exponent after 'p' is decimal, so a trailing 'f' is the binary32 suffix
        named = {k: v.rstrip("f") for k, v in re.findall(r"k(\w+) = (-?0x[0-9a-fp.+-]+)", body)}
        assert F(float.fromhex(named["Ln2Hi"])) == ln2[0]
        assert F(float.fromhex(named["Ln2Lo"])) == ln2[1]
        assert F(float.fromhex(named["Log2e"])) == ln2[2]
        assert F(float.fromhex(named["SqrtHalf"])) == ln2[3]


def _ulps32(got, ref):
    ref = np.asarray(ref, dtype=np.float64)
    return np.abs(got.astype(np.float64) - ref) / np.spacing(np.abs(ref).astype(F32)).astype(
        np.float64)


def test_binary32_accuracy():
    rng = np.random.default_rng(1)
    x = np.concatenate([-rng.uniform(0, 80, 20000), -rng.uniform(0, 1e-3, 500), [0.0, -80.0]])
    x = x.astype(F32)
    xd = x.astype(np.float64)
    assert _ulps32(O.elem("exp", x, F32), np.exp(xd)).max() <= 2
    assert _ulps32(O.elem("expm1", x, F32), np.expm1(xd)).max() <= 2
    y = np.concatenate([rng.uniform(2 ** -24, 1, 20000), rng.uniform(1, 1e6, 2000),
                        [2 ** -24, 0.5, 1.0, 2.0]]).astype(F32)
    lg = O.elem("log", y, F32)
    assert lg[-2] == 0.0  # log 1 = 0 exactly
    err = np.abs(lg.astype(np.float64) - np.log(y.astype(np.float64)))
    assert (err / np.spacing(np.maximum(np.abs(np.log(y.astype(np.float64))), 1e-30).astype(F32))
            .astype(np.float64)).max() <= 2
    z = np.concatenate([rng.uniform(-0.5, 0.5, 20000), [-0.5, 0.0, 1e-30, 0.5]]).astype(F32)
    l1 = O.elem("log1p", z, F32)
    ok = z != 0
    assert _ulps32(l1[ok], np.log1p(z[ok].astype(np.float64))).max() <= 2
    assert l1[~ok].tolist() == [0.0]


def _ulps64_dec(got, ref):
    return max(float(abs(Decimal(float(g)) - r) / Decimal(math.ulp(float(r))))
               for g, r in zip(got, ref))


def test_binary64_accuracy_against_decimal():
    rng = np.random.default_rng(2)
    cases = {"exp": (-rng.uniform(0, 700, 800), lambda d: d.exp()),
             "expm1": (-rng.uniform(0, 40, 800), lambda d: d.exp() - 1),
             "log": (rng.uniform(1e-8, 10, 800), lambda d: d.ln()),
             "log1p": (rng.uniform(-0.5, 0.5, 800), lambda d: (1 + d).ln())}
    for name, (x, ref) in cases.items():
        got = O.elem(name, x, F64)
        assert _ulps64_dec(got, [ref(Decimal(float(v))) for v in x]) <= 2, name


@pytest.mark.parametrize("dtype", [F32, F64])
def test_heat_bath_pass_keeps_the_last_of_k_draws(dtype):
    """A heat-bath draw does not depend on the spin it replaces, so k draws leave the
    last one: the pass's result at every site equals one draw from the site's field
    with the uniforms of draw k - 1 (words 2(k-1) and 2(k-1) + 1 of its stream)."""
    from tests import inputs
    L, seed, k, T, sweep = 4, 61, 3, 0.4, 2
    spins, J = inputs.random_state(L, 9, dtype)
    out = spins.copy()
    O.sweep(L, seed, out, J, T=T, k=k, heat_bath=True, sweep0=sweep)
    col = inputs.colours(L)
    beta = np.dtype(dtype).type(1.0 / T)
    mid = spins.copy()  # state seen by the colour-1 pass: colour 0 already updated
    mid[:, col == 0] = out[:, col == 0]
    for i in range(L ** 3):
        x, y, z = i % L, (i // L) % L, i // (L * L)
        state = spins if col[i] == 0 else mid
        h = O.local_field(L, state, J, x, y, z)
        j = k - 1
        w = O.philox([[sweep, i, j // 2, O.TAG_HB]], seed).ravel()
        u = O.u01(w)
        t = O.heat_bath_draw(h, beta, u[2 * (j % 2)], u[2 * (j % 2) + 1], dtype)
        np.testing.assert_array_equal(out[:, i], t)
