"""The warm-start network's GPU forward and backward passes against the FP64 oracle, and one
training run that lowers the loss."""
import numpy as np
import pytest

from lbm_cases import say
from oracle import mlp as ref

pytestmark = pytest.mark.gpu

DIMS = [4, 128, 128, 128, 64]


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    from paper_1412_5170_amd import lbm
    return lbm, torch


def test_forward_and_gradient_match_fp64_oracle(env):
    lbm, torch = env
    say("[mlp] forward/gradient vs oracle")
    net = lbm.MLP(DIMS, seed=3)
    p = net.get_params().astype(np.float64)
    rng = np.random.default_rng(1)
    for B in (1, 7, 256):
        x = rng.uniform(-1, 1, (B, 4)).astype(np.float32)
        dy = rng.normal(0, 1, (B, 64)).astype(np.float32)
        y = net.forward(torch.from_numpy(x).cuda()).cpu().numpy().astype(np.float64)
        y_ref = ref.forward(p, DIMS, x.astype(np.float64))[-1]
        assert np.max(np.abs(y - y_ref)) <= 1e-5 * max(1.0, np.max(np.abs(y_ref)))
        g = net.gradient(torch.from_numpy(x).cuda(), torch.from_numpy(dy).cuda()).cpu().numpy()
        g_ref = ref.gradient(p, DIMS, x.astype(np.float64), dy.astype(np.float64))
        rel = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
        say(f"    B={B}: forward err {np.max(np.abs(y - y_ref)):.2e}, gradient rel err {rel:.2e}")
        assert rel <= 1e-4
        assert np.max(np.abs(g - g_ref)) <= 1e-4 * np.max(np.abs(g_ref))


def test_training_reduces_loss_deterministically(env):
    lbm, torch = env
    say("[mlp] training")
    rng = np.random.default_rng(2)
    x = torch.from_numpy(rng.uniform(-1, 1, (512, 4)).astype(np.float32)).cuda()
    t = torch.sin(x[:, :1] * 2.0) * torch.linspace(0, 1, 64, device="cuda")[None, :] + x[:, 1:2]
    t = t.contiguous()
    losses = []
    for run in range(2):
        net = lbm.MLP(DIMS, seed=5)
        first = net.train_step(x, t, 1e-3)
        for _ in range(300):
            last = net.train_step(x, t, 1e-3)
        losses.append((first, last, net.get_params()))
    assert losses[0][1] < 0.1 * losses[0][0]
    assert losses[0][1] == losses[1][1] and np.array_equal(losses[0][2], losses[1][2])
