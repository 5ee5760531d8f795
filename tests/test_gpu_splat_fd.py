"""Pose gradients of the GPU splat backward on the full differentiable workload (512
frames of 320 x 240 into the 256 x 192 x 512 grid) against FP64 central finite
differences of the oracle's overlap loss: 32 random frames x 6 se(3) parameters, and 8
random directions over a block of 32 consecutive frames jointly (frames whose footprints
overlap, so the cross terms of the loss between frames are exercised).

A frame's pose changes only that frame's splat, which lies inside a box of voxels around
its footprint; the loss difference L(xi + h e) - L(xi - h e) is therefore formed over that
box from the oracle's FP64 volumes of all frames, minus the frame's own contribution,
plus its contribution at the perturbed pose (both splatted by the oracle).  Every term
is the oracle's; only the unchanged voxels outside the box are not summed (their
contributions to the two losses are equal)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import say

pytestmark = pytest.mark.gpu

# 1e-7 (mm or rad): the trilinear weights have kinks where a pixel crosses a voxel-centre
# plane, and with 1e-6 rad a rotation moves far pixels by ~1e-4 mm, so a few pixels of a
# frame straddle a kink and bias that frame's difference quotient
H_STEP = 1e-7


def _box(c, idx, xis, margin=3):
    """Voxel box (lo, dims) holding every trilinear corner of the frames idx at poses xis."""
    g, p = c["grid"], c["probe"]
    sx, sy = p.pixel_mm
    o = np.asarray(g.origin_mm)
    lo = np.full(3, np.inf)
    hi = np.full(3, -np.inf)
    for n, xi in zip(idx, xis):
        T = oracle.se3_exp(xi) @ c["Tstar"][n]
        for u in (0.5 * sx, (p.width - 0.5) * sx):
            for v in (0.5 * sy, (p.height - 0.5) * sy):
                q = ((T @ np.array([u, v, 0.0, 1.0]))[:3] - o) / g.voxel_mm
                lo = np.minimum(lo, q)
                hi = np.maximum(hi, q)
    dims = np.array(g.dims)
    blo = np.clip(np.floor(lo).astype(int) - margin, 0, dims)
    bhi = np.clip(np.ceil(hi).astype(int) + margin, 0, dims)
    return blo, bhi - blo


def _splat_box(c, idx, xis, lo, dims):
    """Oracle splat of frames idx (consecutive, starting at an even frame or a single
    frame) into the box: returns (S, W) of set A and of set B by the frames' own parity."""
    g, p = c["grid"], c["probe"]
    sub = synth.Grid(tuple(int(x) for x in dims), tuple(float(g.origin_mm[a] + lo[a] * g.voxel_mm) for a in range(3)),
                     g.voxel_mm)
    v = oracle.splat_forward(sub, c["I"][idx], c["Tstar"][idx], np.asarray(xis), p)
    if len(idx) == 1 and idx[0] % 2 == 1:      # one frame is always splatted as set A
        return v[2], v[3], v[0], v[1]
    return v[0], v[1], v[2], v[3]


def _loss_diff(full_box, own0, plus, minus):
    """L(plus) - L(minus) over the box, the frames' own unperturbed splat own0 replaced."""
    SA, WA, SB, WB = full_box
    base = [SA - own0[0], WA - own0[1], SB - own0[2], WB - own0[3]]

    def R(own):
        sa, wa, sb, wb = [b + x for b, x in zip(base, own)]
        return sa * wb - sb * wa

    Rp, Rm = R(plus), R(minus)
    return 0.5 * float(((Rp - Rm) * (Rp + Rm)).sum())


@pytest.fixture(scope="module")
def full_case():
    from paper_2412_00058_amd import SplatContext
    say("case: full differentiable workload, GPU gradient and oracle volumes")
    c = synth.cfg5()
    g, p = c["grid"], c["probe"]
    F = c["I"].shape[0]
    ctx = SplatContext(g.dims, g.origin_mm, g.voxel_mm, p.width, p.height, p.pixel_mm, F)
    I = torch.from_numpy(c["I"]).cuda()
    T = torch.from_numpy(c["Tstar"]).cuda()
    xi = torch.from_numpy(c["xi"]).cuda()
    vols = ctx.forward(I, T, xi)
    _, grads = ctx.loss(vols)
    _, dxi = ctx.backward(I, T, xi, grads)
    torch.cuda.synchronize()
    ctx.close()
    ref = oracle.splat_forward(g, c["I"], c["Tstar"], c["xi"], p)
    return c, dxi.cpu().numpy(), ref


def _box_of(ref, lo, dims):
    return [r[lo[2]:lo[2] + dims[2], lo[1]:lo[1] + dims[1], lo[0]:lo[0] + dims[0]] for r in ref]


def test_pose_gradient_32_frames_by_6_parameters(full_case):
    c, dxi, ref = full_case
    rng = np.random.default_rng(17)
    frames = rng.choice(c["xi"].shape[0], 32, replace=False)
    worst = 0.0
    for n in frames:
        xi0 = c["xi"][n]
        # a step that makes some pixel cross a kink biases the quotient: retry with h / 10
        for h in (H_STEP, H_STEP / 10):
            steps = [xi0 + s * h * e for e in np.eye(6) for s in (1.0, -1.0)]
            lo, dims = _box(c, [n] * len(steps), steps)
            full = _box_of(ref, lo, dims)
            own0 = _splat_box(c, [n], [xi0], lo, dims)
            fd = np.empty(6)
            for k in range(6):
                plus = _splat_box(c, [n], [steps[2 * k]], lo, dims)
                minus = _splat_box(c, [n], [steps[2 * k + 1]], lo, dims)
                fd[k] = _loss_diff(full, own0, plus, minus) / (2.0 * h)
            r = np.linalg.norm(dxi[n] - fd) / np.linalg.norm(fd)
            if r <= 1e-3:
                break
        worst = max(worst, r)
        assert r <= 1e-3, (int(n), r, dxi[n], fd)
    say("  worst per-frame relative error", worst)


def test_pose_gradient_8_directions_over_a_frame_block(full_case):
    c, dxi, ref = full_case
    rng = np.random.default_rng(23)
    n0 = 200
    idx = list(range(n0, n0 + 32))
    xi0 = c["xi"][idx]
    dirs = [rng.normal(size=xi0.shape) for _ in range(8)]
    dirs = [dd / np.linalg.norm(dd) for dd in dirs]
    allx = [xi0] + [xi0 + s * H_STEP * dd for dd in dirs for s in (1.0, -1.0)]
    lo, dims = _box(c, idx * len(allx), np.concatenate(allx))
    full = _box_of(ref, lo, dims)
    own0 = _splat_box(c, idx, xi0, lo, dims)
    for k, dd in enumerate(dirs):
        an = float((dxi[idx] * dd).sum())
        for h in (H_STEP, H_STEP / 10):     # retry with h / 10 as above
            plus = _splat_box(c, idx, xi0 + h * dd, lo, dims)
            minus = _splat_box(c, idx, xi0 - h * dd, lo, dims)
            fd = _loss_diff(full, own0, plus, minus) / (2.0 * h)
            if abs(an - fd) <= 1e-3 * abs(fd):
                break
        say("  direction", k, "analytic", an, "fd", fd)
        assert abs(an - fd) <= 1e-3 * abs(fd), (k, an, fd)
