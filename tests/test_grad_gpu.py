"""GPU parity of the backward kernel (sh_eval_grad) and the autograd op.

Tolerances (per point, g the exact gradient): against the oracle's analytic
gradient |dg|_inf <= 1e-12 (1 + |g|_inf); against central differences of the GPU
forward with h = 1e-6, |dg|_inf <= 1e-7 (1 + |g|_inf)."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import paper_2510_05282_amd as sh
from paper_2510_05282_amd import workloads

pytestmark = pytest.mark.gpu
LD = np.longdouble


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _say(*a):
    print(*a, flush=True)


def _rel_err(got, ref):
    scale = 1 + np.abs(ref.astype(np.float64)).max(axis=1)
    return (np.abs(got.astype(LD) - ref).max(axis=1) / scale).max()


def test_grad_parity_oracle(dev, orc):
    lmax = 6
    pts = np.concatenate([workloads.points_gradient(n=20000, seed=5),
                          np.array([[0, 0, 2.0], [0, 0, -0.7], [1.5, 0, 0], [0, -2, 0],
                                    [1e-9, 0, 1.0], [0, 0, 0.0]])])
    G = np.random.default_rng(6).standard_normal((49, pts.shape[0]))
    _say("case: grad parity lmax 6, n =", pts.shape[0])
    x = torch.from_numpy(pts).to(dev)
    g = sh.sh_eval_grad(lmax, x, torch.from_numpy(G).to(dev)).cpu().numpy()
    ref = orc.grad_xyz(lmax, pts, G)
    err = _rel_err(g, ref)
    _say("  max relative err:", float(err))
    assert err <= 1e-12
    assert np.all(g[-1] == 0)  # the origin


def test_grad_every_lmax(dev, orc):
    pts = workloads.points_gradient(n=3000, seed=7)
    x = torch.from_numpy(pts).to(dev)
    for lmax in range(10):
        _say("case: grad lmax", lmax)
        F = (lmax + 1) ** 2
        G = np.random.default_rng(lmax).standard_normal((F, pts.shape[0]))
        g = sh.sh_eval_grad(lmax, x, torch.from_numpy(G).to(dev)).cpu().numpy()
        assert _rel_err(g, orc.grad_xyz(lmax, pts, G)) <= 1e-12


@pytest.mark.parametrize("n", [1, 63, 65, 257, 1000])
def test_grad_ragged(dev, orc, n):
    pts = workloads.points_gradient(n=n, seed=100 + n)
    G = np.random.default_rng(n).standard_normal((100, n))
    g = sh.sh_eval_grad(9, torch.from_numpy(pts).to(dev), torch.from_numpy(G).to(dev)).cpu().numpy()
    assert _rel_err(g, orc.grad_xyz(9, pts, G)) <= 1e-12


def _fd(dev, lmax, x, G, h=1e-6):
    cols = []
    for k in range(3):
        e = torch.zeros(3, dtype=torch.float64, device=dev)
        e[k] = h
        yp = sh.sh_eval(lmax, (x + e).contiguous())
        ym = sh.sh_eval(lmax, (x - e).contiguous())
        cols.append(((yp - ym) * G).sum(0) / (2 * h))
    return torch.stack(cols, 1)


def test_grad_vs_central_differences(dev):
    lmax = 6
    pts = workloads.points_gradient(n=10000, seed=8)
    x = torch.from_numpy(pts).to(dev)
    G = torch.from_numpy(np.random.default_rng(9).standard_normal((49, 10000))).to(dev)
    g = sh.sh_eval_grad(lmax, x, G)
    fd = _fd(dev, lmax, x, G)
    err = ((g - fd).abs().max(1).values / (1 + g.abs().max(1).values)).max().item()
    _say("  fd max relative err:", err)
    assert err <= 1e-7


def test_grad_full_size_sampled(dev, orc):
    """2^24 points (radius in [0.5, 5]), lmax 6: forward then backward with an
    N(0,1) upstream gradient, in the shape the benchmark times; 10,000 sampled
    points against the oracle's gradient and central differences."""
    n, lmax = 1 << 24, 6
    _say("case: grad full size, n =", n)
    pts = workloads.points_gradient(n=n, seed=0)
    x = torch.from_numpy(pts).to(dev)
    y = sh.sh_eval(lmax, x)
    G = workloads.upstream_gradient_device(49, n, seed=1, device=dev)
    g = sh.sh_eval_grad(lmax, x, G)
    idx = np.sort(np.random.default_rng(2).choice(n, 10000, replace=False))
    it = torch.from_numpy(idx).to(dev)
    gs = g[it].cpu().numpy()
    Gs = G[:, it].contiguous()
    err = _rel_err(gs, orc.grad_xyz(lmax, pts[idx], Gs.cpu().numpy()))
    _say("  oracle max relative err:", float(err))
    assert err <= 1e-12
    fd = _fd(dev, lmax, x[it].contiguous(), Gs).cpu().numpy()
    err_fd = (np.abs(gs - fd).max(1) / (1 + np.abs(gs).max(1))).max()
    _say("  fd max relative err:", float(err_fd))
    assert err_fd <= 1e-7
    del y, G, g


def test_autograd_function(dev):
    pts = workloads.points_gradient(n=5000, seed=10)
    x = torch.from_numpy(pts).to(dev).requires_grad_(True)
    y = sh.spherical_harmonics(x, 5)
    G = torch.from_numpy(np.random.default_rng(11).standard_normal((36, 5000))).to(dev)
    (y * G).sum().backward()
    ref = sh.sh_eval_grad(5, x.detach(), G)
    assert torch.equal(x.grad, ref)
    small = torch.from_numpy(pts[:6]).to(dev).requires_grad_(True)
    assert torch.autograd.gradcheck(lambda t: sh.spherical_harmonics(t, 4), (small,), eps=1e-6,
                                    atol=1e-7, rtol=1e-6)


def test_grad_fp32_parity(dev, orc):
    """FP32 backward against the oracle at the float inputs (upstream gradient in
    float, widened): |dg|_inf <= 2e-5 (1 + |g|_inf)."""
    for lmax in (1, 6, 9):
        pts = workloads.points_gradient(n=20000, seed=30 + lmax).astype(np.float32)
        F = (lmax + 1) ** 2
        G = np.random.default_rng(lmax).standard_normal((F, pts.shape[0])).astype(np.float32)
        g = sh.sh_eval_grad_f32(lmax, torch.from_numpy(pts).to(dev), torch.from_numpy(G).to(dev))
        ref = orc.grad_xyz(lmax, pts.astype(np.float64), G.astype(np.float64))
        err = _rel_err(g.cpu().numpy(), ref)
        _say("  fp32 grad lmax", lmax, "max relative err:", float(err))
        assert err <= 2e-5
        # and against the FP64 backward kernel on the same GPU at the same inputs
        g64 = sh.sh_eval_grad(lmax, torch.from_numpy(pts.astype(np.float64)).to(dev),
                              torch.from_numpy(G.astype(np.float64)).to(dev))
        assert _rel_err(g.cpu().numpy(), g64.cpu().numpy()) <= 2e-5


@pytest.mark.parametrize("extra", [0, 1])
def test_fused_values_and_jacobian(dev, orc, extra):
    """5003 points (odd: one point per lane) and 5004 (two points per lane)."""
    pts = np.concatenate([workloads.points_gradient(n=5000, seed=40),
                          np.array([[0, 0, 1.5], [0, 0, 0.0], [2.0, 0, 0]]),
                          np.array([[0.3, -0.2, 0.1]])[:extra]])
    origin = int(np.flatnonzero(np.all(pts == 0, axis=1))[0])
    for lmax in (0, 3, 9):
        F = (lmax + 1) ** 2
        y, j = sh.sh_eval_jac(lmax, torch.from_numpy(pts).to(dev))
        y, j = y.cpu().numpy(), j.cpu().numpy()
        assert np.abs(y.astype(LD) - orc.eval_xyz(lmax, pts)).max() <= 1e-13
        J = orc.jacobian_xyz(lmax, pts)
        scale = 1 + np.abs(J.astype(np.float64)).max()
        assert np.abs(j.astype(LD) - J).max() <= 1e-12 * scale
        assert np.all(j[:, :, origin] == 0)
        assert y.shape == (F, pts.shape[0])


def test_autograd_fp32(dev):
    pts = workloads.points_gradient(n=3000, seed=12).astype(np.float32)
    x = torch.from_numpy(pts).to(dev).requires_grad_(True)
    y = sh.spherical_harmonics(x, 4)
    assert y.dtype == torch.float32
    G = torch.from_numpy(np.random.default_rng(13).standard_normal((25, 3000)).astype(np.float32)).to(dev)
    (y * G).sum().backward()
    assert torch.equal(x.grad, sh.sh_eval_grad_f32(4, x.detach(), G))


@pytest.mark.parametrize("n", [6000, 6003])
@pytest.mark.parametrize("lmax", [4, 12, 24])
def test_grad_by_recurrence(dev, orc, lmax, n):
    """Backward pass up to l = 24 (differentiated recurrence) against the oracle's
    analytic gradient (FP64 1e-12 (1 + |g|), FP32 2e-5 / 5e-6 (lmax + 1)), against
    central differences of the GPU forward, and through torch autograd.  n + 1
    points (the last at the origin): 6001 takes the one-point-per-lane launch,
    6004 the two-point one."""
    F = (lmax + 1) ** 2
    pts = np.concatenate([workloads.points_gradient(n=n, seed=50 + lmax), np.zeros((1, 3))])
    G = np.random.default_rng(lmax).standard_normal((F, pts.shape[0]))
    x, Gt = torch.from_numpy(pts).to(dev), torch.from_numpy(G).to(dev)
    g = sh.sh_eval_grad_rec(lmax, x, Gt).cpu().numpy()
    assert _rel_err(g, orc.grad_xyz(lmax, pts, G)) <= 1e-12
    assert np.all(g[-1] == 0)  # origin
    if lmax <= 9:
        assert _rel_err(g, sh.sh_eval_grad(lmax, x, Gt).cpu().numpy().astype(LD)) <= 1e-12
    h = 1e-6
    fd = np.zeros_like(g)
    for k in range(3):
        e = torch.zeros(3, dtype=torch.float64, device=dev)
        e[k] = h
        yp = sh.sh_eval_rec(lmax, (x + e).contiguous())
        ym = sh.sh_eval_rec(lmax, (x - e).contiguous())
        fd[:, k] = ((yp - ym) / (2 * h) * Gt).sum(0).cpu().numpy()
    scale = 1 + np.abs(g).max(axis=1)
    assert (np.abs(fd[:-1] - g[:-1]).max(axis=1) / scale[:-1]).max() <= 1e-6
    xr = x.clone().requires_grad_(True)
    (sh.spherical_harmonics(xr, lmax) * Gt).sum().backward()
    assert torch.equal(xr.grad, torch.from_numpy(g).to(dev) if lmax > 9 else sh.sh_eval_grad(lmax, x, Gt))
    p32, G32 = pts.astype(np.float32), G.astype(np.float32)
    g32 = sh.sh_eval_grad_rec_f32(lmax, torch.from_numpy(p32).to(dev), torch.from_numpy(G32).to(dev)).cpu().numpy()
    ref32 = orc.grad_xyz(lmax, p32.astype(np.float64), G32.astype(np.float64))
    assert _rel_err(g32, ref32) <= (2e-5 if lmax <= 9 else 5e-6 * (lmax + 1))
