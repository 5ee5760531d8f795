"""GPU trilinear splat, overlap loss and hand-written backward against the FP64 oracle:
forward within rel 1e-5 (norm-wise), gradients within rel 1e-3 of FP64 central
differences of the oracle's loss, through the C ABI and through torch.autograd."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import say

pytestmark = pytest.mark.gpu


def ctx_for(c):
    from paper_2412_00058_amd import SplatContext
    g, p = c["grid"], c["probe"]
    return SplatContext(g.dims, g.origin_mm, g.voxel_mm, p.width, p.height, p.pixel_mm, c["I"].shape[0])


def dev(c):
    return (torch.from_numpy(c["I"]).cuda(), torch.from_numpy(c["Tstar"]).cuda(), torch.from_numpy(c["xi"]).cuda())


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def check_forward(c, tol=1e-5):
    ctx = ctx_for(c)
    I, T, xi = dev(c)
    vols = ctx.forward(I, T, xi).cpu().numpy().astype(np.float64)
    ref = oracle.splat_forward(c["grid"], c["I"], c["Tstar"], c["xi"], c["probe"])
    for k in range(4):
        r = rel(vols[k], ref[k].ravel())
        say("  volume", k, "rel", r)
        assert r <= tol, (k, r)
    return ctx, vols, ref


def test_forward_small_and_reduced_cfg5():
    say("case: small splat forward")
    check_forward(synth.small_splat())
    say("case: cfg5 64 frames forward")
    check_forward(synth.cfg5(n_frames=64, dims=(256, 192, 64)))


def test_forward_dense_pixels_take_the_direct_path():
    # 0.02 mm pixels in 0.5 mm voxels: about 7,600 pixels of one frame can reach a voxel,
    # too many for the 32-bit fixed-point window, so the tiles add their terms with FP32
    # global atomics; same tolerance against the FP64 oracle
    say("case: dense pixels, direct forward path")
    c = synth.cfg5(n_frames=6, W=120, H=96, px=0.02, dims=(8, 8, 6))
    c["I"] = np.random.default_rng(8).uniform(-1.0, 1.0, c["I"].shape).astype(np.float32)
    check_forward(c)


def test_forward_unit_cases():
    say("case: voxel-centre pixels")
    F, H, W = 4, 6, 7
    g = np.random.default_rng(2)
    I = g.uniform(0, 1, (F, H, W)).astype(np.float32)
    T = np.stack([np.eye(4) for _ in range(F)])
    for n in range(F):
        T[n, 2, 3] = 0.25 + 0.5 * (n % 3)
    c = dict(I=I, Tstar=T, xi=np.zeros((F, 6)), probe=synth.Probe(W, H, (0.5, 0.5)),
             grid=synth.Grid((8, 8, 4), (0, 0, 0), 0.5))
    ctx = ctx_for(c)
    vols = ctx.forward(*dev(c)).cpu().numpy()
    ref = oracle.splat_forward(c["grid"], I, T, c["xi"], c["probe"])
    assert np.array_equal(vols[1], ref[1].ravel().astype(np.float32))       # W_A exact counts
    assert np.abs(vols[0] - ref[0].ravel()).max() < 1e-6


def test_loss_and_gradients_vs_fp64_finite_differences():
    say("case: small splat gradients")
    c = synth.small_splat()
    ctx = ctx_for(c)
    I, T, xi = dev(c)
    vols = ctx.forward(I, T, xi)
    loss, grads = ctx.loss(vols)
    dI, dxi = ctx.backward(I, T, xi, grads)
    dI, dxi = dI.cpu().numpy(), dxi.cpu().numpy()
    vols64 = oracle.splat_forward(c["grid"], c["I"], c["Tstar"], c["xi"], c["probe"])
    L64, G64 = oracle.overlap_loss(vols64)
    assert abs(float(loss.item()) - L64) <= 1e-4 * abs(L64)

    def Lxi(x):
        return oracle.overlap_loss(oracle.splat_forward(c["grid"], c["I"], c["Tstar"], x, c["probe"]), False)

    F = c["xi"].shape[0]
    h = 1e-6
    fd = np.zeros((F, 6))
    for n in range(F):
        for j in range(6):
            xp, xm = c["xi"].copy(), c["xi"].copy()
            xp[n, j] += h
            xm[n, j] -= h
            fd[n, j] = (Lxi(xp) - Lxi(xm)) / (2 * h)
    for n in range(F):
        r = np.linalg.norm(dxi[n] - fd[n]) / np.linalg.norm(fd[n])
        assert r <= 1e-3, (n, r, dxi[n], fd[n])
    dI64, dxi64 = oracle.splat_backward(c["grid"], c["I"], c["Tstar"], c["xi"], c["probe"], G64)
    assert rel(dI, dI64) <= 1e-3
    # intensities: central differences of the FP64 loss at sampled pixels (quadratic in I)
    g = np.random.default_rng(1)
    for _ in range(10):
        n, v, u = g.integers(0, F), g.integers(0, c["I"].shape[1]), g.integers(0, c["I"].shape[2])
        hh = 2.0 ** -8
        Ip, Im = c["I"].astype(np.float64).copy(), c["I"].astype(np.float64).copy()
        Ip[n, v, u] += hh
        Im[n, v, u] -= hh
        lp = oracle.overlap_loss(oracle.splat_forward(c["grid"], Ip.astype(np.float32), c["Tstar"], c["xi"],
                                                      c["probe"]), False)
        lm = oracle.overlap_loss(oracle.splat_forward(c["grid"], Im.astype(np.float32), c["Tstar"], c["xi"],
                                                      c["probe"]), False)
        fdI = (lp - lm) / (2 * hh)
        assert abs(dI[n, v, u] - fdI) <= 1e-3 * (abs(fdI) + 1e-3 * np.abs(dI64).max())


def test_autograd_matches_direct_calls():
    from paper_2412_00058_amd import OverlapLossFn, SplatFn
    say("case: autograd")
    c = synth.small_splat()
    ctx = ctx_for(c)
    I, T, xi = dev(c)
    I.requires_grad_(True)
    xi.requires_grad_(True)
    vols = SplatFn.apply(ctx, I, xi, T)
    L = OverlapLossFn.apply(ctx, vols)
    L.backward()
    v2 = ctx.forward(I.detach(), T, xi.detach())
    l2, g2 = ctx.loss(v2)
    dI2, dxi2 = ctx.backward(I.detach(), T, xi.detach(), g2)
    # FP32 atomics make two forward passes differ in the last bits (run-to-run spread)
    assert abs(L.item() - l2.item()) <= 1e-6 * abs(l2.item())
    assert rel(I.grad.cpu().numpy(), dI2.cpu().numpy()) <= 1e-5
    assert rel(xi.grad.cpu().numpy(), dxi2.cpu().numpy()) <= 1e-5


def test_full_cfg5_forward_and_gradient_vs_oracle():
    say("case: cfg5 full size")
    c = synth.cfg5()
    ctx, vols, ref = check_forward(c)
    I, T, xi = dev(c)
    loss, grads = ctx.loss(torch.from_numpy(vols.astype(np.float32)).cuda())
    dI, dxi = ctx.backward(I, T, xi, grads)
    L64, G64 = oracle.overlap_loss(ref)
    assert abs(loss.item() - L64) <= 1e-4 * abs(L64)
    dI64, dxi64 = oracle.splat_backward(c["grid"], c["I"], c["Tstar"], c["xi"], c["probe"], G64)
    dxi = dxi.cpu().numpy()
    g = np.random.default_rng(3)
    for n in g.choice(c["xi"].shape[0], 32, replace=False):
        r = np.linalg.norm(dxi[n] - dxi64[n]) / np.linalg.norm(dxi64[n])
        assert r <= 1e-3, (n, r)
    assert rel(dI.cpu().numpy(), dI64) <= 1e-3
    # one global random direction by FP64 central differences of the oracle loss
    dirn = g.normal(size=c["xi"].shape)
    dirn /= np.linalg.norm(dirn)
    h = 1e-6
    lp = oracle.overlap_loss(oracle.splat_forward(c["grid"], c["I"], c["Tstar"], c["xi"] + h * dirn, c["probe"]), False)
    lm = oracle.overlap_loss(oracle.splat_forward(c["grid"], c["I"], c["Tstar"], c["xi"] - h * dirn, c["probe"]), False)
    fd = (lp - lm) / (2 * h)
    an = float((dxi * dirn).sum())
    assert abs(an - fd) <= 1e-3 * abs(fd), (an, fd)
