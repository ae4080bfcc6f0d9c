"""The structured allocation forms the GPU step uses, checked on the CPU in
FP64 against the oracle's allocation matrix and its min-norm pseudo-inverse
(reading R12 of the layouts): for the quad X layout, A^+ and A are one +-1
pattern scaled per row, so both products are 4-point butterflies; for the
hexa and octo layouts, rotor i + n/2 sits opposite rotor i, so its rows are
rotor i's with the x-y terms negated and the yaw term times (-1)^(n/2), and
the products run over opposite pairs.  These restate the forms in numpy
(independent of the HIP code) so that a wrong sign or index in a form fails
here before any GPU run.
"""
import numpy as np
import pytest
import torch

from oracle import allocation

ARMS = [0.05, 0.13, 1.5]
CTAUS = [1e-3, 0.016, 0.3]


def pinv_and_a(n, arm, ctau):
    A = allocation.allocation_matrix(n, torch.tensor([arm], dtype=torch.float64),
                                     torch.tensor([ctau], dtype=torch.float64))[0].numpy()
    return np.linalg.pinv(A), A


def quad_butterflies(f, M, arm, ctau, clamp):
    # scales of the unit-arm A^+ (c_f, c_x, c_z) and A (s, c_tau)
    cf, cx, cz = 0.25, np.sqrt(0.5) / 2 / arm, 1.0 / (4 * ctau)
    a, b = cf * f + cz * M[2], cf * f - cz * M[2]
    c, d = cx * M[0] - cx * M[1], cx * M[0] + cx * M[1]
    u = clamp(np.array([a + c, b + d, a - c, b - d]))
    e, o, ge, ho = u[0] + u[2], u[1] + u[3], u[0] - u[2], u[1] - u[3]
    s = np.sqrt(0.5) * arm
    return u, np.array([e + o, s * (ge + ho), s * (ho - ge), ctau * (e - o)])


def pair_form(n, f, M, pinv, A, clamp):
    h = n // 2
    zs = pinv[0, 3] * M[2]
    cp, cm = pinv[0, 0] * f + zs, pinv[0, 0] * f - zs
    u = np.zeros(n)
    for i in range(h):
        L = pinv[i, 1] * M[0] + pinv[i, 2] * M[1]
        sp = i % 2 == 0
        so = (not sp) if h % 2 else sp
        u[i] = (cp if sp else cm) + L
        u[i + h] = (cp if so else cm) - L
    u = clamp(u)
    fa = x0 = x1 = yaw = 0.0
    for i in range(h):
        d, sm = u[i] - u[i + h], u[i] + u[i + h]
        fa += sm
        x0 += A[1, i] * d
        x1 += A[2, i] * d
        yaw += (1 if i % 2 == 0 else -1) * (d if h % 2 else sm)
    return u, np.array([fa, x0, x1, A[3, 0] * yaw])


@pytest.mark.parametrize("n", [4, 6, 8])
@pytest.mark.parametrize("arm", ARMS)
@pytest.mark.parametrize("ctau", CTAUS)
def test_structured_forms_equal_pseudo_inverse_and_matrix(n, arm, ctau):
    rng = np.random.default_rng(n * 1000 + int(arm * 100) + int(ctau * 1e4))
    pinv, A = pinv_and_a(n, arm, ctau)
    # the structure the forms rely on, in exact arithmetic (FP64 to 1e-12)
    h = n // 2
    for i in range(h):
        o = i + h
        assert np.allclose(pinv[o, :3], pinv[i, :3] * [1, -1, -1], atol=1e-12 * abs(pinv).max())
        assert np.isclose(pinv[o, 3], pinv[i, 3] * (-1) ** h)
        assert np.allclose(A[:3, o], A[:3, i] * [1, -1, -1], atol=1e-12)
        assert np.isclose(A[3, o], A[3, i] * (-1) ** h)
    umax = 24.0 / n
    for clamp in (lambda u: u, lambda u: np.clip(u, 0.0, umax)):
        for _ in range(20):
            f = rng.uniform(0, 30)
            M = rng.uniform(-1, 1, 3) * [arm * 5, arm * 5, ctau * 20]
            u_ref = clamp(pinv @ np.concatenate([[f], M]))
            w_ref = A @ u_ref
            if n == 4:
                u, w = quad_butterflies(f, M, arm, ctau, clamp)
            else:
                # the pair form takes the unit-arm rows (M_x, M_y divided by l)
                # and the A rows with the arm factored out, as the kernel does
                p1 = pinv.copy()
                p1[:, 1:3] *= arm
                a1 = A.copy()
                a1[1:3] /= arm
                u, w = pair_form(n, f, np.array([M[0] / arm, M[1] / arm, M[2]]), p1, a1, clamp)
                w = w * np.array([1, arm, arm, 1])
            assert np.allclose(u, u_ref, rtol=1e-12, atol=1e-12 * umax)
            assert np.allclose(w, w_ref, rtol=1e-12, atol=1e-10)
