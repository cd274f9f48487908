"""Cost-model kernels against the fp64 oracle: forward, gradient (checked
against the oracle's backpropagation, itself pinned by central differences)
and the Adam step.  fp32 tolerance: each output is a sum of at most
D*H + H*H + H products of O(1) terms, so its rounding error stays below
~1e-5 relative; 1e-4 relative plus 1e-6 of the largest entry is asserted."""
import numpy as np
import pytest

from oracle import mlp as ref

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mj():
    import paper_1504_07038_amd as mj

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    mj.lib()
    return mj


def close(got, exp, rtol=1e-4):
    got = np.asarray(got, dtype=np.float64)
    exp = np.asarray(exp, dtype=np.float64)
    tol = rtol * np.abs(exp) + 1e-6 * max(1.0, np.max(np.abs(exp)))
    return np.all(np.abs(got - exp) <= tol), np.max(np.abs(got - exp) / (np.abs(exp) + 1e-30))


def f32(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.mark.parametrize("D,H,N", [(5, 16, 1), (9, 32, 37), (16, 32, 1000), (3, 16, 8193)])
def test_forward_and_gradient_match_oracle(mj, D, H, N):
    rng = np.random.default_rng(D * 100 + H + N)
    p = ref.init(D, H, seed=N).astype(np.float32).astype(np.float64)
    p += rng.normal(0, 0.05, len(p))
    p = p.astype(np.float32).astype(np.float64)        # both sides see the same fp32 values
    x = rng.normal(0, 1, (N, D)).astype(np.float32).astype(np.float64)
    t = rng.normal(0, 1, N).astype(np.float32).astype(np.float64)
    assert mj.mojette_mlp_params(D, H) == ref.nparams(D, H) == len(p)
    d_p, d_x, d_t = f32(p), f32(x), f32(t)
    d_y = torch.empty(N, dtype=torch.float32, device="cuda")
    mj.mojette_mlp_forward(d_p, D, H, d_x, d_y)
    ws = torch.empty(mj.mojette_mlp_grad_workspace(D, H, N), dtype=torch.float32, device="cuda")
    d_g = torch.empty(len(p) + 1, dtype=torch.float32, device="cuda")
    mj.mojette_mlp_grad(d_p, D, H, d_x, d_t, d_g, ws)
    torch.cuda.synchronize()
    ok, err = close(d_y.cpu().numpy(), ref.forward(p, x, D, H))
    assert ok, err
    g, L = ref.grad(p, x, t, D, H)
    got = d_g.cpu().numpy()
    ok, err = close(got[:-1], g, rtol=2e-4)
    assert ok, err
    assert abs(got[-1] - L) <= 1e-4 * L + 1e-7
    # reproducible bit for bit
    d_g2 = torch.empty_like(d_g)
    mj.mojette_mlp_grad(d_p, D, H, d_x, d_t, d_g2, ws)
    torch.cuda.synchronize()
    assert torch.equal(d_g, d_g2)


def test_adam_step_matches_oracle(mj):
    rng = np.random.default_rng(5)
    n = 1234
    p = rng.normal(size=n).astype(np.float32)
    m = (rng.normal(size=n) * 0.1).astype(np.float32)
    v = (rng.random(n) * 0.01).astype(np.float32)
    g = rng.normal(size=n).astype(np.float32)
    d_p, d_m, d_v, d_g = f32(p), f32(m), f32(v), f32(g)
    mj.mojette_mlp_adam(d_p, d_g, d_m, d_v, 1e-3, 0.9, 0.999, 1e-8, 7)
    torch.cuda.synchronize()
    ep, em, ev = ref.adam(p.astype(np.float64), g.astype(np.float64), m, v, 7, 1e-3, 0.9, 0.999, 1e-8)
    for got, exp in ((d_p, ep), (d_m, em), (d_v, ev)):
        ok, err = close(got.cpu().numpy(), exp, rtol=1e-5)
        assert ok, err


def test_training_fits_a_smooth_function(mj):
    """Full-batch Adam on the GPU kernels fits y = sin(x0) + x1 * x2 well
    below the variance of the target (a sanity check of the loop)."""
    rng = np.random.default_rng(9)
    D, H, N = 3, 32, 4096
    x = rng.uniform(-1.5, 1.5, (N, D))
    t = np.sin(x[:, 0]) + x[:, 1] * x[:, 2]
    d_x, d_t = f32(x), f32(t)
    d_p = f32(ref.init(D, H, seed=1))
    d_m = torch.zeros_like(d_p)
    d_v = torch.zeros_like(d_p)
    d_g = torch.empty(d_p.numel() + 1, dtype=torch.float32, device="cuda")
    ws = torch.empty(mj.mojette_mlp_grad_workspace(D, H, N), dtype=torch.float32, device="cuda")
    for step in range(1, 801):
        mj.mojette_mlp_grad(d_p, D, H, d_x, d_t, d_g, ws)
        mj.mojette_mlp_adam(d_p, d_g[:-1], d_m, d_v, 3e-3, 0.9, 0.999, 1e-8, step)
    torch.cuda.synchronize()
    mj.mojette_mlp_grad(d_p, D, H, d_x, d_t, d_g, ws)
    torch.cuda.synchronize()
    assert float(d_g[-1]) < 0.02 * float(np.var(t))
