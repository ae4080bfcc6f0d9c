"""The sine/cosine form the GPU step uses for command angles, restated in
numpy FP32 (fused multiply-adds evaluated in FP64 and rounded once more to
FP32) and checked against numpy's FP64 sin and cos: Cody-Waite reduction by
pi/2 with a three-part split of pi/2, Taylor polynomials of degree 9 and 10
on [-pi/4, pi/4], and the quadrant of k.  A wrong split part, coefficient,
quadrant swap or sign fails the error bound here before any GPU run; the GPU
parity tests then compare the kernels' wrenches, which depend on these
values, with the FP64 oracle.
"""
import numpy as np

F32 = np.float32
PIO2 = (F32(float.fromhex("0x1.921fb6p+0")), F32(float.fromhex("-0x1.777a5cp-25")),
        F32(float.fromhex("-0x1.ee59dap-50")))
TWO_OVER_PI = F32(float.fromhex("0x1.45f306p-1"))
SIN_C = [F32(float.fromhex(h)) for h in ("0x1.71de3ap-19", "-0x1.a01a02p-13", "0x1.111112p-7", "-0x1.555556p-3")]
COS_C = [F32(float.fromhex(h)) for h in ("-0x1.27e4fcp-22", "0x1.a01a02p-16", "-0x1.6c16c2p-10",
                                         "0x1.555556p-5", "-0x1p-1")]


def fma(a, b, c):
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(F32)


def sincos_form(x):
    x = np.asarray(x, F32)
    k = np.rint(x * TWO_OVER_PI).astype(F32)
    r = fma(-k, np.full_like(x, PIO2[0]), x)
    r = fma(-k, np.full_like(x, PIO2[1]), r)
    r = fma(-k, np.full_like(x, PIO2[2]), r)
    r2 = r * r
    ps = fma(np.full_like(x, SIN_C[0]), r2, np.full_like(x, SIN_C[1]))
    ps = fma(ps, r2, np.full_like(x, SIN_C[2]))
    ps = fma(ps, r2, np.full_like(x, SIN_C[3]))
    ps = ps * r2
    pc = fma(np.full_like(x, COS_C[0]), r2, np.full_like(x, COS_C[1]))
    for c in COS_C[2:]:
        pc = fma(pc, r2, np.full_like(x, c))
    sr = np.where(x == 0, x, fma(r, ps, r))
    cr = fma(pc, r2, np.ones_like(x))
    q = (k + F32(1.5 * 2.0 ** 23)).view(np.int32) & 3     # k mod 4 from the float's low bits
    odd = (q & 1) == 1
    s = np.where(odd, cr, sr)
    c = np.where(odd, sr, cr)
    s = np.where((q & 2) != 0, -s, s)
    c = np.where(((q + 1) & 2) != 0, -c, c)
    return s, c


def test_split_and_coefficients_are_what_they_claim():
    # the three parts add up to pi/2 within the FP32 spacing of the last one
    tot = sum(float(p) for p in PIO2)
    assert abs(tot - np.pi / 2) < 1e-22
    import math
    for c, n in zip(SIN_C, (9, 7, 5, 3)):
        assert abs(abs(float(c)) - 1 / math.factorial(n)) <= np.spacing(F32(1 / math.factorial(n)))
    for c, n in zip(COS_C, (10, 8, 6, 4, 2)):
        assert abs(abs(float(c)) - 1 / math.factorial(n)) <= np.spacing(F32(1 / math.factorial(n)))


def test_error_bound_over_the_fast_range():
    rng = np.random.default_rng(0)
    x = np.concatenate([
        rng.uniform(-np.pi, np.pi, 400_000),
        rng.uniform(-4095.0, 4095.0, 400_000),
        # close to multiples of pi/2, where the reduced argument cancels
        (np.arange(-2600, 2600) * (np.pi / 2))[:, None] + np.array([-1e-5, -1e-7, 0.0, 1e-7, 1e-5])[None, :],
    ], axis=None).astype(F32)
    s, c = sincos_form(x)
    xd = x.astype(np.float64)
    es = np.abs(s.astype(np.float64) - np.sin(xd))
    ec = np.abs(c.astype(np.float64) - np.cos(xd))
    # an absolute bound of 1.5 FP32 ulps of 1 (values are in [-1, 1])
    assert es.max() < 1.8e-7, es.max()
    assert ec.max() < 1.8e-7, ec.max()


def test_zero_and_quadrant_signs():
    s, c = sincos_form(np.array([0.0, -0.0], F32))
    assert s[0] == 0 and not np.signbit(s[0]) and np.signbit(s[1]) and np.all(c == 1)
    # one point inside each quadrant, both signs of x
    x = np.array([0.3, 1.9, 3.5, 5.0, -0.3, -1.9, -3.5, -5.0], F32)
    s, c = sincos_form(x)
    assert np.array_equal(np.sign(s), np.sign(np.sin(x.astype(np.float64))))
    assert np.array_equal(np.sign(c), np.sign(np.cos(x.astype(np.float64))))
