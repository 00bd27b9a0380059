"""Clearance cost and its hand-written gradient on the GPU against the
float64 oracle and float64 central differences (relative tolerance 1e-4)."""
import numpy as np
import pytest
import torch

import oracle
from oracle import clearance as cl
import workloads
from paper_2105_04419_amd import ClearanceCost, Field

pytestmark = pytest.mark.gpu
H, MARGIN = 0.2, 1.0


@pytest.fixture(scope="module")
def field():
    assert torch.cuda.is_available()
    occ = workloads.dense_boxes(0)
    f = Field((64, 64, 32), 20)
    f.global_(torch.from_numpy(occ).cuda())
    s_gpu = f.dense()
    s_ref = oracle.edt_separable(occ, 20)
    assert np.array_equal(s_gpu.cpu().numpy(), s_ref)
    return occ, s_gpu, s_ref


def tol_ok(g, gref, rel=1e-4):
    scale = np.abs(gref).max()
    return np.abs(g - gref) <= rel * np.maximum(np.abs(gref), 1e-3 * scale)


def test_forward_matches_fp64(field):
    occ, s_gpu, s_ref = field
    wp = workloads.trajectories(0, occ, ntraj=512)
    c = ClearanceCost.apply(s_gpu, torch.from_numpy(wp).cuda(), H, MARGIN).cpu().numpy()
    ref = cl.cost(s_ref, wp, H, MARGIN)
    assert np.all(np.abs(c - ref) <= 1e-5 * np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max()) + 1e-6)


def test_backward_matches_fp64_analytic(field):
    occ, s_gpu, s_ref = field
    wp = workloads.trajectories(1, occ, ntraj=4096)
    x = torch.from_numpy(wp).cuda().requires_grad_(True)
    c = ClearanceCost.apply(s_gpu, x, H, MARGIN)
    gc = torch.linspace(0.5, 2.0, c.numel(), device="cuda")
    (c * gc).sum().backward()
    g = x.grad.cpu().numpy().astype(np.float64)
    gref = cl.cost_grad(s_ref, wp, H, MARGIN, gc.cpu().numpy().astype(np.float64))
    ok = tol_ok(g, gref)
    assert ok.all(), f"{(~ok).sum()} components outside tolerance"


def test_backward_matches_central_differences(field):
    occ, s_gpu, s_ref = field
    wp = workloads.trajectories(2, occ, ntraj=256)
    x = torch.from_numpy(wp).cuda().requires_grad_(True)
    ClearanceCost.apply(s_gpu, x, H, MARGIN).sum().backward()
    g = x.grad.cpu().numpy().astype(np.float64)
    w64 = wp.astype(np.float64)
    eps = 1e-4
    gfd = cl.cost_grad_fd(s_ref, w64, H, MARGIN, eps)
    u = w64 / H
    frac = u - np.floor(u)
    d, gd = cl.trilinear(cl.metric_field(s_ref, H), w64, H)
    near = (np.minimum(frac, 1 - frac) < 10 * eps / H) | \
           (np.abs(MARGIN - d) < 10 * eps * np.linalg.norm(gd, axis=-1))[..., None]
    ok = tol_ok(g, gfd) | near
    bad = np.argwhere(~ok)
    assert len(bad) == 0, (f"{len(bad)} components differ from central differences, first "
                           f"{bad[0].tolist()}: {g[tuple(bad[0])]} vs {gfd[tuple(bad[0])]}"
                           if len(bad) else "")


def test_zero_cost_far_from_obstacles_and_clamped_axes(field):
    occ, s_gpu, s_ref = field
    s = torch.full((8, 8, 8), 400, dtype=torch.int32, device="cuda")
    wp = torch.rand(3, 5, 3, device="cuda") * 1.4
    x = wp.clone().requires_grad_(True)
    c = ClearanceCost.apply(s, x, H, MARGIN)
    c.sum().backward()
    assert (c == 0).all() and (x.grad == 0).all()
    # outside the grid along x: the x component of the gradient is zero
    wp2 = torch.tensor([[[-1.0, 0.33, 0.41], [20.0, 0.5, 0.7]]], device="cuda")
    x2 = wp2.clone().requires_grad_(True)
    ClearanceCost.apply(s_gpu, x2, H, MARGIN).sum().backward()
    assert (x2.grad[..., 0] == 0).all()


def test_deterministic(field):
    occ, s_gpu, _ = field
    wp = torch.from_numpy(workloads.trajectories(3, occ, ntraj=1024)).cuda()
    a = ClearanceCost.apply(s_gpu, wp, H, MARGIN)
    b = ClearanceCost.apply(s_gpu, wp, H, MARGIN)
    assert torch.equal(a, b)
