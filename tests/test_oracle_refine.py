"""Pins of the oracle's rigid-motion refinement (Adam over one se(3) motion of the odd
frames against the overlap loss), independent of the HIP path:
  * Adam's first step from zero moments is x - lr g / (|g| + eps) (closed form), and Adam
    on a separable quadratic reaches its minimiser;
  * on a two-pass case whose second pass was taken after a known rigid patient motion
    (built from rotation matrices, not from the se(3) exponential), the refinement
    recovers that motion: Exp(xi) delta^-1 is the identity to 0.05 mm and 0.1 deg, from a
    start 1.1 mm / 1.1 deg away.  A wrong sign, frame set or composition order in the loss,
    the pose gradient or the update cannot pass this."""
import math

import numpy as np

import oracle
import synth


def test_adam_first_step_closed_form():
    g = np.array([3.0, -0.5, 1e-3, -7.0, 2.0, 0.25])
    x0 = np.linspace(-1.0, 1.0, 6)
    lr = np.array([0.1, 0.1, 0.1, 0.01, 0.01, 0.01])
    x1, m, v = oracle.adam_step(x0, g, np.zeros(6), np.zeros(6), 1, lr, 0.9, 0.999, 1e-8)
    np.testing.assert_allclose(x1, x0 - lr * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-14)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-14)


def test_adam_reaches_quadratic_minimum():
    c = np.array([0.3, -1.2, 2.0])
    w = np.array([1.0, 10.0, 0.1])          # badly scaled on purpose: Adam is per-component
    x, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    for t in range(1, 3001):
        x, m, v = oracle.adam_step(x, w * (x - c), m, v, t, 0.01)
    np.testing.assert_allclose(x, c, atol=1e-3)


def residual(xi, delta):
    E = oracle.se3_exp(xi) @ np.linalg.inv(delta)
    ang = math.degrees(math.acos(min(1.0, (np.trace(E[:3, :3]) - 1.0) / 2.0)))
    return float(np.linalg.norm(E[:3, 3])), ang


def test_refinement_recovers_patient_motion():
    c = synth.two_pass_case(n_frames=48, W=64, H=48, px=0.5, spacing=0.3, voxel=0.75, n_blobs=8)
    t0, a0 = residual(np.zeros(6), c["delta"])
    assert t0 > 1.0 and a0 > 1.0
    xi, L = oracle.refine_motion(c["grid"], c["I"], c["Tstar"], c["probe"], iters=150, lr_rho=0.1,
                                 lr_omega=math.radians(0.1))
    t1, a1 = residual(xi, c["delta"])
    assert t1 < 0.05 and a1 < 0.1, (t1, a1)
    assert L.shape == (151,) and L[-1] < 0.01 * L[0]
    # posing the odd frames at the true motion gives the same low loss
    Ltrue = oracle.overlap_loss(oracle.splat_forward(c["grid"], c["I"], c["Ttrue"], np.zeros((48, 6)), c["probe"]),
                                want_grads=False)
    assert abs(L[-1] - Ltrue) < 0.1 * L[-1] + 1e-9, (L[-1], Ltrue)
