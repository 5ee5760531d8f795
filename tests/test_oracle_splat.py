"""Pins of the oracle's se(3) maps, trilinear splat, overlap loss and gradients (the
differentiable addition beside the paper's PNN path): library matrix exponential,
complex-step derivatives, closed-form weights, partition of unity, adjointness and
central finite differences."""
import math

import numpy as np
import pytest
from scipy.linalg import expm

import oracle
import synth


def hat(xi):
    X = np.zeros((4, 4), dtype=np.result_type(xi, np.float64))
    r, w = xi[:3], xi[3:]
    X[:3, :3] = [[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]]
    X[:3, 3] = r
    return X


def vee(X):
    return np.array([X[0, 3], X[1, 3], X[2, 3], X[2, 1], X[0, 2], X[1, 0]])


@pytest.mark.parametrize("scale", [1e-6, 0.02, 0.7, 2.5])
def test_se3_exp_matches_expm(scale):
    g = np.random.default_rng(int(scale * 1000) + 1)
    xi = g.normal(size=6) * scale
    xi[:3] *= 30.0
    assert np.abs(oracle.se3_exp(xi) - expm(hat(xi))).max() <= 1e-12 * (1 + np.abs(xi).max())


@pytest.mark.parametrize("scale", [0.0, 0.02, 0.5, 2.0])
def test_left_jacobian_matches_complex_step(scale):
    # J_l(xi) e_j = vee( dExp(xi + t e_j)/dt  Exp(xi)^-1 ), derivative by complex step
    g = np.random.default_rng(int(scale * 100) + 7)
    xi = g.normal(size=6) * scale
    xi[:3] *= 10.0
    J = oracle.se3_left_jacobian(xi)
    E_inv = np.linalg.inv(expm(hat(xi)))
    h = 1e-30
    for j in range(6):
        xc = xi.astype(np.complex128)
        xc[j] += 1j * h
        dE = np.imag(expm(hat(xc))) / h
        col = vee(dE @ E_inv)
        assert np.abs(col - J[:, j]).max() <= 1e-12 * (1 + np.abs(J).max()), (j, col, J[:, j])


def _probe(W, H, px):
    return synth.Probe(W, H, (px, px))


def test_voxel_centres_reduce_to_nearest_tally():
    # pixel centres exactly on voxel centres: f = 0, all weight on one voxel
    g = np.random.default_rng(2)
    F, H, W = 4, 6, 7
    I = g.uniform(0, 1, (F, H, W)).astype(np.float32)
    T = np.stack([np.eye(4) for _ in range(F)])
    for n in range(F):
        T[n, 2, 3] = 0.25 + 0.5 * (n % 3)      # z on voxel centres; frames 0 and 3 coincide
    grid = synth.Grid((8, 8, 4), (0.0, 0.0, 0.0), 0.5)
    SA, WA, SB, WB = oracle.splat_forward(grid, I, T, np.zeros((F, 6)), _probe(W, H, 0.5))
    wantS = [np.zeros((4, 8, 8)), np.zeros((4, 8, 8))]
    wantW = [np.zeros((4, 8, 8)), np.zeros((4, 8, 8))]
    for n in range(F):
        z = n % 3
        wantS[n % 2][z, :H, :W] += I[n]
        wantW[n % 2][z, :H, :W] += 1.0
    assert np.abs(SA - wantS[0]).max() < 1e-12 and np.abs(SB - wantS[1]).max() < 1e-12
    assert np.array_equal(WA, wantW[0]) and np.array_equal(WB, wantW[1])


def test_single_pixel_weights_by_hand():
    # one pixel at voxel coordinate p = q - 1/2 = (1.25, 2.5, 0.75): i0 = (1, 2, 0), f = (.25, .5, .75)
    s = 0.5
    T = np.eye(4)
    T[:3, 3] = np.array([1.75, 3.0, 1.25]) * s - np.array([0.5, 0.5, 0.0]) * 1.0
    I = np.array([[[2.0]]], np.float32)
    grid = synth.Grid((4, 4, 4), (0.0, 0.0, 0.0), s)
    SA, WA, SB, WB = oracle.splat_forward(grid, I, T[None], np.zeros((1, 6)), _probe(1, 1, 1.0))
    f = (0.25, 0.5, 0.75)
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                w = (f[0] if dx else 1 - f[0]) * (f[1] if dy else 1 - f[1]) * (f[2] if dz else 1 - f[2])
                assert abs(WA[0 + dz, 2 + dy, 1 + dx] - w) < 1e-15
                assert abs(SA[0 + dz, 2 + dy, 1 + dx] - 2.0 * w) < 1e-15
    assert abs(WA.sum() - 1.0) < 1e-15 and SB.sum() == 0 and WB.sum() == 0


def test_partition_of_unity_inside_grid():
    c = synth.small_splat()
    grid, probe = c["grid"], c["probe"]
    big = synth.Grid((48, 40, 24), (-4.0, -4.0, -2.0), 0.5)
    SA, WA, SB, WB = oracle.splat_forward(big, c["I"], c["Tstar"], c["xi"], probe)
    F, H, W = c["I"].shape
    assert abs(WA.sum() + WB.sum() - F * H * W) < 1e-8
    assert abs(SA.sum() + SB.sum() - c["I"].astype(np.float64).sum()) < 1e-8


def test_adjoint_identity():
    # <Splat_S(I), G> = <I, dL/dI> when G_S = G and G_W = 0 (the slice is the adjoint)
    c = synth.small_splat()
    g = np.random.default_rng(12)
    shape = c["grid"].dims[::-1]
    GA, GB = g.normal(size=shape), g.normal(size=shape)
    SA, WA, SB, WB = oracle.splat_forward(c["grid"], c["I"], c["Tstar"], c["xi"], c["probe"])
    Z = np.zeros(shape)
    dI, _ = oracle.splat_backward(c["grid"], c["I"], c["Tstar"], c["xi"], c["probe"], [GA, Z, GB, Z])
    lhs = (SA * GA).sum() + (SB * GB).sum()
    rhs = (c["I"].astype(np.float64) * dI).sum()
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_overlap_loss_closed_form():
    SA, WA, SB, WB = [np.array([1.0, 2.0, 0.0]), np.array([2.0, 1.0, 0.0]),
                      np.array([3.0, 0.0, 5.0]), np.array([1.0, 0.0, 2.0])]
    L, G = oracle.overlap_loss([SA, WA, SB, WB])
    R = np.array([1 * 1 - 3 * 2, 0.0, 0.0])
    assert L == 0.5 * (R ** 2).sum()
    assert np.array_equal(G[0], R * WB) and np.array_equal(G[3], R * SA)
    assert np.array_equal(G[2], -R * WA) and np.array_equal(G[1], -R * SB)


def _loss(c, xi, I):
    vols = oracle.splat_forward(c["grid"], I, c["Tstar"], xi, c["probe"])
    return oracle.overlap_loss(vols, want_grads=False)


def test_gradients_match_central_differences():
    c = synth.small_splat()
    xi, I = c["xi"], c["I"]
    vols = oracle.splat_forward(c["grid"], I, c["Tstar"], xi, c["probe"])
    L0, G = oracle.overlap_loss(vols)
    dI, dxi = oracle.splat_backward(c["grid"], I, c["Tstar"], xi, c["probe"], G)
    F = xi.shape[0]
    h = 1e-6
    worst = 0.0
    for n in range(F):
        for j in range(6):
            best = None
            for hh in (h, h / 10):
                xp, xm = xi.copy(), xi.copy()
                xp[n, j] += hh
                xm[n, j] -= hh
                fd = (_loss(c, xp, I) - _loss(c, xm, I)) / (2 * hh)
                err = abs(fd - dxi[n, j]) / (abs(dxi[n]).max() + 1e-12)
                best = err if best is None else min(best, err)
            worst = max(worst, best)
    assert worst <= 1e-5, worst
    # intensities: the loss is quadratic in I -> central differences are exact up to rounding
    g = np.random.default_rng(3)
    for _ in range(12):
        n, v, u = g.integers(0, F), g.integers(0, I.shape[1]), g.integers(0, I.shape[2])
        Ip, Im = I.astype(np.float64).copy(), I.astype(np.float64).copy()
        hh = 2.0 ** -10
        Ip[n, v, u] += hh
        Im[n, v, u] -= hh
        vp = oracle.splat_forward(c["grid"], Ip.astype(np.float32), c["Tstar"], xi, c["probe"])
        vm = oracle.splat_forward(c["grid"], Im.astype(np.float32), c["Tstar"], xi, c["probe"])
        fd = (oracle.overlap_loss(vp, False) - oracle.overlap_loss(vm, False)) / (2 * hh)
        assert abs(fd - dI[n, v, u]) <= 1e-6 * (1 + abs(dI).max())
