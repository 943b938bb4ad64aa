"""Cost-model network kernels on the GPU against the float64 oracle:
inference, the mean-squared-error gradient (relative error <= 1e-4) and
Adam; plus a short training run that must reduce the loss."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1907_06487_amd import _lib
from oracle import mlp as M

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
U32 = 2.0 ** -24


def _theta(seed, scale=0.3):
    return (M.init_params(seed) + scale * np.random.default_rng(seed).normal(size=M.N_PARAMS)).astype(np.float32)


def _abs_net(theta, X):
    p = M.unpack(np.abs(theta.astype(np.float64)))
    h1 = np.abs(X) @ p["W1"].T + p["b1"]
    h2 = h1 @ p["W2"].T + p["b2"]
    return h2 @ p["w3"] + p["b3"][0]


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device=DEV)


@pytest.mark.parametrize("n", [1, 255, 1000, 70001])
def test_forward_matches_oracle(n):
    print(f"case mlp forward n={n}", flush=True)
    theta = _theta(n % 7)
    X = np.random.default_rng(n).normal(size=(n, 12)).astype(np.float32)
    y = torch.full((n,), float("nan"), dtype=torch.float32, device=DEV)
    _lib.race_mlp_forward(_dev(theta), _dev(X), y)
    torch.cuda.synchronize()
    ref = M.forward(theta.astype(np.float64), X.astype(np.float64))
    bound = 3 * 66 * U32 * _abs_net(theta, X.astype(np.float64))
    assert np.all(np.abs(y.cpu().numpy() - ref) <= bound)


def _grad_gpu(theta, X, t):
    n = X.shape[0]
    ws = torch.empty(_lib.race_mlp_workspace(n), dtype=torch.float32, device=DEV)
    g = torch.full((M.N_PARAMS,), float("nan"), dtype=torch.float32, device=DEV)
    loss = torch.full((1,), float("nan"), dtype=torch.float32, device=DEV)
    _lib.race_mlp_loss_grad(_dev(theta), _dev(X), _dev(t), ws, g, loss)
    torch.cuda.synchronize()
    return g.cpu().numpy().astype(np.float64), float(loss.item())


@pytest.mark.parametrize("n", [1, 255, 256, 257, 5000])
def test_gradient_matches_oracle(n):
    print(f"case mlp gradient n={n}", flush=True)
    theta = _theta(3 + n % 5)
    rng = np.random.default_rng(100 + n)
    X = rng.normal(size=(n, 12)).astype(np.float32)
    t = rng.normal(size=n).astype(np.float32)
    g, loss = _grad_gpu(theta, X, t)
    ref_loss, ref = M.loss_and_grad(theta.astype(np.float64), X.astype(np.float64), t.astype(np.float64))
    rel = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    print(f"  gradient relative error {rel:.2e}, loss {loss:.6g} vs {ref_loss:.6g}", flush=True)
    assert rel <= 1e-4
    assert abs(loss - ref_loss) <= 1e-5 * ref_loss
    for block in ("W1", "b1", "W2", "b2", "w3", "b3"):  # every block, not only the largest
        gb, rb = M.unpack(g)[block], M.unpack(ref)[block]
        assert np.linalg.norm(gb - rb) <= 1e-4 * np.linalg.norm(ref) + 1e-12


def test_gradient_is_deterministic():
    theta = _theta(11)
    rng = np.random.default_rng(12)
    X = rng.normal(size=(3000, 12)).astype(np.float32)
    t = rng.normal(size=3000).astype(np.float32)
    g1, l1 = _grad_gpu(theta, X, t)
    g2, l2 = _grad_gpu(theta, X, t)
    assert np.array_equal(g1, g2) and l1 == l2


@pytest.mark.parametrize("steps", [1, 2, 10])
def test_adam_matches_oracle(steps):
    rng = np.random.default_rng(20 + steps)
    theta = rng.normal(size=M.N_PARAMS).astype(np.float32)
    grads = [rng.normal(size=M.N_PARAMS).astype(np.float32) for _ in range(steps)]
    th, m, v = _dev(theta), torch.zeros(M.N_PARAMS, device=DEV), torch.zeros(M.N_PARAMS, device=DEV)
    ref_t, ref_m, ref_v = theta.astype(np.float64), np.zeros(M.N_PARAMS), np.zeros(M.N_PARAMS)
    # the kernel receives the hyperparameters as float32: give the oracle the
    # same (rounded) values, e.g. 1 - float32(0.999) = 0.00099998713
    f32 = lambda a: float(np.float32(a))
    for s, g in enumerate(grads, start=1):
        _lib.race_mlp_adam(th, _dev(g), m, v, s, 1e-2)
        ref_t, ref_m, ref_v = M.adam_step(ref_t, g.astype(np.float64), ref_m, ref_v, s, f32(1e-2), beta1=f32(0.9),
                                          beta2=f32(0.999), eps=f32(1e-8))
    torch.cuda.synchronize()
    assert np.allclose(th.cpu().numpy(), ref_t, rtol=1e-5, atol=1e-6)
    assert np.allclose(m.cpu().numpy(), ref_m, rtol=1e-5, atol=1e-7)
    assert np.allclose(v.cpu().numpy(), ref_v, rtol=1e-5, atol=1e-9)


def test_training_reduces_loss():
    """Fit a random teacher network from a fresh start with the device
    kernels only: the loss must fall by more than 10x."""
    rng = np.random.default_rng(30)
    teacher = _theta(31, 0.1).astype(np.float64)
    X = rng.normal(size=(4096, 12))
    t = M.forward(teacher, X)
    Xd, td = _dev(X.astype(np.float32)), _dev(t.astype(np.float32))
    th = _dev(M.init_params(32).astype(np.float32))
    m, v = torch.zeros(M.N_PARAMS, device=DEV), torch.zeros(M.N_PARAMS, device=DEV)
    ws = torch.empty(_lib.race_mlp_workspace(512), dtype=torch.float32, device=DEV)
    g = torch.empty(M.N_PARAMS, dtype=torch.float32, device=DEV)
    loss = torch.empty(1, dtype=torch.float32, device=DEV)
    ws_all = torch.empty(_lib.race_mlp_workspace(4096), dtype=torch.float32, device=DEV)
    g_all = torch.empty_like(g)
    _lib.race_mlp_loss_grad(th, Xd, td, ws_all, g_all, loss)
    torch.cuda.synchronize()
    first = loss.item()
    step = 0
    for epoch in range(40):
        order = torch.randperm(4096, device=DEV)
        for b in range(0, 4096, 512):
            idx = order[b:b + 512]
            step += 1
            _lib.race_mlp_loss_grad(th, Xd[idx].contiguous(), td[idx].contiguous(), ws, g, loss)
            _lib.race_mlp_adam(th, g, m, v, step, 3e-3)
    _lib.race_mlp_loss_grad(th, Xd, td, ws_all, g_all, loss)
    torch.cuda.synchronize()
    last = loss.item()
    print(f"training loss {first:.4g} -> {last:.4g} after {step} steps", flush=True)
    assert last < first / 10
