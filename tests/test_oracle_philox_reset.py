"""Pins of the oracle's Philox4x32-10 (against rocRAND's host-side engine, an
independent implementation of the same published generator) and of the
reset draw, mask and compaction."""
import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
import torch

from oracle import philox, reset, so3

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_ref():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND reference")
    d = tempfile.mkdtemp(prefix="philox_ref_")
    exe = os.path.join(d, "ref")
    subprocess.run([hipcc, "-x", "hip", "--offload-host-only", "-O1",
                    os.path.join(HERE, "rocrand_philox_ref.cpp"), "-o", exe], check=True)

    def run(ctr, key):
        lines = "\n".join(" ".join(str(int(v)) for v in list(c) + list(k)) for c, k in zip(ctr, key))
        out = subprocess.run([exe], input=lines, capture_output=True, text=True, check=True).stdout
        return np.array([[int(w) for w in ln.split()] for ln in out.strip().splitlines()], np.uint64)

    yield run
    shutil.rmtree(d, ignore_errors=True)


def test_philox_matches_rocrand(rocrand_ref):
    rng = np.random.default_rng(0)
    n = 400
    ctr = rng.integers(0, 2 ** 32, size=(n, 4), dtype=np.uint64)
    ctr[:, 1] %= 2 ** 30        # the reference reaches counter word 1 through a 64-bit offset
    key = rng.integers(0, 2 ** 32, size=(n, 2), dtype=np.uint64)
    ctr[:4] = 0
    key[:2] = 0
    ours = philox.philox4x32_10(ctr, key).astype(np.uint64)
    ref = rocrand_ref(ctr, key)
    assert np.array_equal(ours, ref)


def test_mask_rate_is_binomial():
    n, p = 200_000, 0.01
    idx = np.arange(n)
    hits = sum(int(reset.mask(idx, t, 12345, p).sum()) for t in range(5))
    mean, sd = 5 * n * p, math.sqrt(5 * n * p * (1 - p))
    assert abs(hits - mean) < 5 * sd
    assert reset.threshold(0.01) == 42_949_672
    assert reset.mask(idx[:10], 3, 1, 0.0).sum() == 0
    assert reset.mask(idx[:10], 3, 1, 1.0).all()


def test_mask_depends_only_on_global_index_and_step():
    """Sharding invariance: a vehicle's decision is the same in any batch."""
    idx = np.arange(10_000)
    full = reset.mask(idx, 17, 99, 0.05)
    part = reset.mask(idx[4000:6000], 17, 99, 0.05)
    assert np.array_equal(full[4000:6000], part)
    assert not np.array_equal(reset.mask(idx, 18, 99, 0.05), full)


def test_reset_draws_and_compaction():
    n = 5000
    st = torch.zeros(n, 13, dtype=torch.float64)
    st[:, 6] = 1.0
    tg = torch.zeros(n, 4, dtype=torch.float64)
    tg[:, 3] = 0.7
    mode = np.where(np.arange(n) % 3 == 0, 0, 1)
    s2, t2, m, idx = reset.apply(st, mode, tg, np.arange(n), 41, 7, 0.2, (-5, -5, -5), (5, 5, 5))
    assert idx.dtype == np.int32
    assert np.array_equal(idx, np.flatnonzero(m))
    assert np.all(np.diff(idx) > 0)
    keep = ~m
    assert torch.equal(s2[keep], st[keep]) and torch.equal(t2[keep], tg[keep])
    r = s2[idx]
    assert (r[:, 0:3].abs() <= 5).all()
    assert ((r[:, 6:10].norm(dim=-1) - 1).abs() < 1e-14).all()
    R = so3.quat_to_rot(r[:, 6:10])
    tilt = torch.acos(R[:, 2, 2].clamp(-1, 1))
    assert (tilt <= math.pi / 6 + 1e-12).all()
    pos = mode[idx] == 0
    assert (t2[idx][pos, 3] == 0).all() and (t2[idx][~pos, 3] == 0.7).all()
    assert (t2[idx][pos, :3].abs() <= 5).all()
    # uniform words map exactly onto 24-bit grids
    w = reset.draw_words(idx[:50], 41, 7)
    u = (w >> 8).astype(np.float64) * 2.0 ** -24
    assert np.array_equal(u.astype(np.float32).astype(np.float64), u)


def test_reset_tilt_equals_drawn_angle():
    """q = qz(psi) (x) q_axis(tau): the angle between b3 and e3 is exactly tau."""
    idx = np.arange(64)
    w = reset.draw_words(idx, 5, 3)
    u = (w >> 8).astype(np.float64) * 2.0 ** -24
    s, _ = reset.redraw(idx, 5, 3, (-1, -1, -1), (1, 1, 1))
    R = so3.quat_to_rot(s[:, 6:10])
    tilt = torch.acos(R[:, 2, 2].clamp(-1, 1)).numpy()
    np.testing.assert_allclose(tilt, reset.TILT_MAX * u[:, 7], atol=1e-7)


def _uniform_rows(k):
    u = np.full((k, 16), 0.5)
    return u


def test_redraw_normals_closed_form():
    """Box-Muller on chosen uniforms: with 1 - u_a = e^(-1/2) the radius is
    exactly 1, with u_a = 3/4 it is sqrt(2 ln 4) (it would be sqrt(-2 ln 3/4)
    with ln u_a), and u_a = 0 gives 0; the angle 2 pi u_b puts the radius on
    the first normal of the pair for u_b = 0 and on the second for u_b = 1/4.
    Pair (9, 10) -> v_x, v_y; (11, 12) -> v_z, Omega_x; (13, 14) -> Omega_y,
    Omega_z; velocity sigma 0.5, rate sigma 0.2."""
    one = 1.0 - math.exp(-0.5)
    u = _uniform_rows(5)
    u[0, 9], u[0, 10] = one, 0.0           # v = (0.5, 0, .)
    u[1, 9], u[1, 10] = one, 0.25          # v = (0, 0.5, .)
    u[2, 9], u[2, 10] = 0.75, 0.5          # v_x = -0.5 sqrt(2 ln 4)
    u[3, 9] = 0.0                          # r = 0
    u[0, 11], u[0, 12] = one, 0.0          # v_z = 0.5, Omega_x = 0
    u[1, 11], u[1, 12] = one, 0.25         # v_z = 0, Omega_x = 0.2
    u[0, 13], u[0, 14] = one, 0.125        # Omega_y = Omega_z = 0.2 / sqrt 2
    u[1, 13], u[1, 14] = 0.75, 0.75        # Omega_z = -0.2 sqrt(2 ln 4)
    s, _ = reset.state_from_uniforms(u, (-1, -1, -1), (1, 1, 1))
    s = s.numpy()
    r4 = math.sqrt(2.0 * math.log(4.0))
    tol = 1e-15
    assert abs(s[0, 3] - 0.5) < tol and abs(s[0, 4]) < tol
    assert abs(s[1, 3]) < tol and abs(s[1, 4] - 0.5) < tol
    assert abs(s[2, 3] + 0.5 * r4) < tol and abs(s[2, 4]) < 1e-15
    assert s[3, 3] == 0.0 and s[3, 4] == 0.0
    assert abs(s[0, 5] - 0.5) < tol and abs(s[0, 10]) < tol
    assert abs(s[1, 5]) < tol and abs(s[1, 10] - 0.2) < tol
    assert abs(s[0, 11] - 0.2 / math.sqrt(2)) < tol and abs(s[0, 12] - 0.2 / math.sqrt(2)) < tol
    assert abs(s[1, 11]) < tol and abs(s[1, 12] + 0.2 * r4) < tol


def test_redraw_normals_statistics():
    """On 200,000 Philox draws the velocity and rate components are N(0, 0.5^2)
    and N(0, 0.2^2): sample mean within 5 standard errors of 0, sample sigma
    within 5 standard errors (sigma / sqrt(2n)) of sigma, a Kolmogorov-Smirnov
    test against the normal CDF, and the two normals of one Box-Muller pair
    uncorrelated.  Positions and tilt are uniform on their ranges (KS)."""
    from scipy import stats as st
    n = 200_000
    s, goal = reset.redraw(np.arange(n), 3, 11, (-5, -4, -3), (5, 4, 3))
    s = s.numpy()
    for cols, sigma in (((3, 4, 5), 0.5), ((10, 11, 12), 0.2)):
        for c in cols:
            x = s[:, c]
            assert abs(x.mean()) < 5 * sigma / math.sqrt(n)
            assert abs(x.std() - sigma) < 5 * sigma / math.sqrt(2 * n)
            assert st.kstest(x, "norm", args=(0.0, sigma)).pvalue > 1e-4
    rho = np.corrcoef(s[:, 3], s[:, 4])[0, 1]
    assert abs(rho) < 5 / math.sqrt(n)
    for d, h in enumerate((5, 4, 3)):
        assert st.kstest(s[:, d], "uniform", args=(-h, 2 * h)).pvalue > 1e-4
        assert st.kstest(goal.numpy()[:, d], "uniform", args=(-h, 2 * h)).pvalue > 1e-4
    R = so3.quat_to_rot(torch.as_tensor(s[:, 6:10]))
    tilt = torch.acos(R[:, 2, 2].clamp(-1, 1)).numpy()
    assert st.kstest(tilt, "uniform", args=(0.0, reset.TILT_MAX)).pvalue > 1e-4
