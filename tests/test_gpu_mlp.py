"""The learned-schedule kernels against the FP64 reference MLP (needs an MI355X)."""
import numpy as np
import pytest
import torch

from oracle import mlp as M
from paper_2205_12182_amd import _lib as L

pytestmark = pytest.mark.gpu


def dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def setup_case(nout, B, seed=0):
    rng = np.random.default_rng(seed)
    p = M.init_params(nout, seed=seed) + 0.02 * rng.standard_normal(M.param_count(nout))
    p = p.astype(np.float32).astype(np.float64)           # what the GPU sees
    x = rng.standard_normal((B, M.NIN)).astype(np.float32).astype(np.float64)
    t = rng.standard_normal((B, nout)).astype(np.float32).astype(np.float64)
    return p, x, t


@pytest.mark.parametrize("nout,B", [(1, 1000), (2, 333), (4, 64)])
def test_forward_backward_against_reference(gpu_ok, nout, B):
    assert L.nolsm_mlp_param_count(nout) == M.param_count(nout)
    p, x, t = setup_case(nout, B)
    P = M.param_count(nout)
    dp, dx, dt = dev(p), dev(x), dev(t)
    y = torch.empty(B, nout, device="cuda")
    act = torch.empty(B, 2 * M.NH, device="cuda")
    L.nolsm_mlp_forward(dp, nout, dx, y, act)
    dy = torch.empty_like(y)
    loss = torch.empty(1, device="cuda")
    scratch = torch.empty(L.nolsm_mlp_scratch_floats(B, nout), device="cuda")
    L.nolsm_mlp_mse(y, dt, dy, loss, scratch)
    grad = torch.empty(P, device="cuda")
    L.nolsm_mlp_backward(dp, nout, dx, act, dy, grad, scratch)
    torch.cuda.synchronize()
    yr, cache = M.forward(p, nout, x)
    lr_, dyr = M.mse(yr, t)
    gr = M.backward(p, nout, x, cache, dyr)
    assert np.abs(y.cpu().numpy() - yr).max() <= 1e-5 * (1 + np.abs(yr).max())
    assert abs(loss.item() - lr_) <= 1e-5 * lr_
    g = grad.cpu().numpy()
    # relative error of the gradient, per parameter block and overall (FP32 kernels)
    assert np.linalg.norm(g - gr) <= 1e-3 * np.linalg.norm(gr)
    big = np.abs(gr) > 1e-3 * np.abs(gr).max()
    assert np.all(np.abs(g[big] - gr[big]) <= 1e-3 * np.abs(gr[big]) + 1e-6 * np.abs(gr).max())


def test_backward_is_deterministic(gpu_ok):
    p, x, t = setup_case(1, 5000, seed=4)
    dp, dx, dt = dev(p), dev(x), dev(t)
    y = torch.empty(5000, 1, device="cuda")
    act = torch.empty(5000, 2 * M.NH, device="cuda")
    dy = torch.empty_like(y)
    loss = torch.empty(1, device="cuda")
    scratch = torch.empty(L.nolsm_mlp_scratch_floats(5000, 1), device="cuda")
    grads = []
    for _ in range(2):
        L.nolsm_mlp_forward(dp, 1, dx, y, act)
        L.nolsm_mlp_mse(y, dt, dy, loss, scratch)
        g = torch.empty(M.param_count(1), device="cuda")
        L.nolsm_mlp_backward(dp, 1, dx, act, dy, g, scratch)
        grads.append(g)
    assert torch.equal(grads[0], grads[1])


def test_adam_step_against_reference(gpu_ok):
    rng = np.random.default_rng(1)
    P = 333
    p = rng.standard_normal(P).astype(np.float32)
    g = rng.standard_normal(P).astype(np.float32)
    m = (0.1 * rng.standard_normal(P)).astype(np.float32)
    v = np.abs(0.1 * rng.standard_normal(P)).astype(np.float32)
    dp, dg, dm, dv = dev(p), dev(g), dev(m), dev(v)
    L.nolsm_mlp_adam(dp, dg, dm, dv, 1e-3, 0.9, 0.999, 1e-8, 7)
    pr, mr, vr = M.adam(p.astype(np.float64), g, m, v, 1e-3, 0.9, 0.999, 1e-8, 7)
    assert np.allclose(dp.cpu().numpy(), pr, atol=1e-6, rtol=1e-5)
    assert np.allclose(dm.cpu().numpy(), mr, atol=1e-7, rtol=1e-5)
    assert np.allclose(dv.cpu().numpy(), vr, atol=1e-7, rtol=1e-5)


def test_training_reduces_loss(gpu_ok):
    from paper_2205_12182_amd.learn import ScheduleMLP
    rng = np.random.default_rng(0)
    x = rng.standard_normal((4096, M.NIN)).astype(np.float32)
    t = np.tanh(x[:, :3] @ np.array([1.0, -0.7, 0.4]))[:, None].astype(np.float32)
    net = ScheduleMLP(nout=1, seed=3)
    hist = net.fit(x, t, steps=400, lr=3e-3)
    assert hist[-1] < 0.05 * hist[0]


def reference_features(Mk, n, nmem, m, mu):
    """The 16 descriptors written out from their definitions (A = M_k - mu I, n x n)."""
    A = Mk[:n, :n].astype(np.float64) - mu * np.eye(n)
    d = np.diag(A)
    R = np.abs(A).sum(axis=0) - np.abs(d)
    f2 = (A * A).sum()
    b = np.max(np.abs(d) + R)
    mean, rms = d.mean(), np.sqrt(f2 / n)
    var = max((d * d).mean() - mean * mean, 0.0)
    mind = np.abs(d).min()
    return np.array([np.log(n), nmem / 100.0, m / 32.0, np.log(b), (d - R).min() / b,
                     (d + R).max() / b, mean / b, rms / b, np.sqrt(var) / b, mind / b,
                     R.sum() / n / b, R.max() / b, (d < 0).mean(), np.abs(d).mean() / b,
                     mind / rms, 1.0])


def test_features_match_definition(gpu_ok):
    """nolsm_features (two passes over M_k, partials combined in column order) against
    the descriptors computed in FP64 from the same FP32 M_k read back."""
    from paper_2205_12182_amd import learn
    from paper_2205_12182_amd.runner import Runner
    from workloads import get_config
    inst = get_config("t_slab")
    r = Runner(inst)
    L.nolsm_build_submatrices(r.plans[0], r.dpat, r.H, r.S)
    feat = learn.features(r, 0, inst.mu).cpu().numpy()
    for i in [0, 7, inst.nmol // 2, inst.nmol - 1]:
        info = r.sub_info(0, i)
        Mk = r.ws_view(info.off_h, info.npad * info.npad, torch.float32).reshape(
            info.npad, info.npad).T.cpu().numpy()
        ref = reference_features(Mk, info.n, info.nmem, info.m, inst.mu)
        assert np.allclose(feat[i], ref, rtol=2e-6, atol=2e-6), (i, feat[i], ref)
