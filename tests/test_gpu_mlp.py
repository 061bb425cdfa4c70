"""The network kernels (through the C ABI) against the FP64 oracle.

The oracle receives the bfloat16-rounded weights the GPU multiplies with, so
the remaining differences are FP32 activations and accumulation: forward and
gradients agree to 1e-4 relative; Adam to 1e-6.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import mlp as om

pytestmark = pytest.mark.gpu


def say(m):
    print(m, flush=True)
    sys.stdout.flush()


def _data(seed, B):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((B, 64)).astype(np.float32)
    y = (rng.random(B) < 0.5).astype(np.float32)
    return x, y


@pytest.mark.parametrize("B", [1, 31, 32, 100, 1000])
def test_forward_matches_oracle(gpu, B):
    say(f"mlp forward B={B}")
    import torch
    from paper_2609_12476_amd.mlp import Mlp
    p = synth.mlp_init_params(1)
    p[om.N_PARAMS - 1] = 0.25
    net = Mlp(max_batch=1024, params=p)
    x, _ = _data(2, B)
    z = net.forward(torch.from_numpy(x).to(gpu)).cpu().numpy().astype(np.float64)
    zr, _ = om.forward(om.weights_as_used(p), x)
    assert np.max(np.abs(z - zr)) <= 1e-4 * max(1.0, np.max(np.abs(zr)))
    net.close()


@pytest.mark.parametrize("B", [1, 64, 257])
def test_gradient_matches_oracle(gpu, B):
    say(f"mlp gradient B={B}")
    import torch
    from paper_2609_12476_amd.mlp import Mlp
    p = synth.mlp_init_params(3)
    net = Mlp(max_batch=512, params=p)
    x, y = _data(4, B)
    g, loss = net.gradient(torch.from_numpy(x).to(gpu), torch.from_numpy(y).to(gpu))
    g = g.cpu().numpy().astype(np.float64)
    lr, gr = om.loss_and_grad(om.weights_as_used(p), x, y)
    assert abs(float(loss.cpu()) - lr) <= 1e-5 * max(1.0, abs(lr))
    # per block of parameters, relative l2
    o = 0
    for name, shape in om.SHAPES:
        n = int(np.prod(shape))
        a, b = g[o:o + n], gr[o:o + n]
        nb = np.linalg.norm(b)
        assert np.linalg.norm(a - b) <= 1e-4 * nb + 1e-9, name
        o += n
    net.close()


def test_gradient_is_deterministic(gpu):
    import torch
    from paper_2609_12476_amd.mlp import Mlp
    net = Mlp(max_batch=512, params=synth.mlp_init_params(5))
    x, y = _data(6, 300)
    xt, yt = torch.from_numpy(x).to(gpu), torch.from_numpy(y).to(gpu)
    g1, _ = net.gradient(xt, yt)
    g2, _ = net.gradient(xt, yt)
    assert torch.equal(g1, g2)
    net.close()


def test_adam_matches_oracle(gpu):
    say("mlp adam")
    import torch
    from paper_2609_12476_amd.mlp import Mlp
    p = synth.mlp_init_params(7)
    net = Mlp(max_batch=8, params=p)
    rng = np.random.default_rng(8)
    pr, m, v = p.astype(np.float64), np.zeros(om.N_PARAMS), np.zeros(om.N_PARAMS)
    for t in range(1, 4):
        g = (rng.standard_normal(om.N_PARAMS) * 1e-2).astype(np.float32)
        net.adam_step(torch.from_numpy(g).to(gpu), 1e-3)
        pr, m, v = om.adam(pr, m, v, g, t, 1e-3)
    got = net.get_params().astype(np.float64)
    assert np.max(np.abs(got - pr)) <= 1e-6 * max(1.0, np.max(np.abs(pr)))
    net.close()


def test_training_reduces_loss_on_separable_data(gpu):
    say("mlp training")
    import torch
    from paper_2609_12476_amd.mlp import Mlp
    rng = np.random.default_rng(9)
    B = 512
    x = rng.standard_normal((4096, 64)).astype(np.float32)
    y = (x[:, :8].sum(axis=1) > 0).astype(np.float32)
    net = Mlp(max_batch=B, params=synth.mlp_init_params(10))
    xt, yt = torch.from_numpy(x).to(gpu), torch.from_numpy(y).to(gpu)
    loss = torch.empty(1, device=gpu)
    first = None
    for it in range(200):
        i = (it * B) % 4096
        net.train_step(xt[i:i + B], yt[i:i + B], 1e-3, loss)
        if first is None:
            first = float(loss.cpu())
    z = net.forward(xt).cpu().numpy()
    acc = np.mean((z > 0) == (y > 0.5))
    say(f"  first loss {first:.3f}, accuracy {acc:.3f}")
    assert float(loss.cpu()) < 0.5 * first and acc > 0.95
    net.close()


def test_region_features_match_definition(gpu):
    say("region features")
    import torch
    from paper_2609_12476_amd.mlp import nr_mlp_region_features
    rng = np.random.default_rng(11)
    n_mc, n_sub, K, L = 9, 3, 30, 7680
    stat = (rng.gamma(50.0, L, size=(n_mc * n_sub, K))).astype(np.float32)
    stat[4, 17] *= 3
    used = rng.integers(0, 60, size=n_mc * n_sub).astype(np.int32)
    used[5] = 0
    f = nr_mlp_region_features(torch.from_numpy(stat.ravel()).to(gpu), torch.from_numpy(used).to(gpu),
                               n_mc, n_sub, K, 1.0 / L).cpu().numpy()
    for region in range(n_mc * n_sub):
        mc, sb = divmod(region, n_sub)
        ks = int(np.argmax(stat[region]))
        for i in range(8):
            m2 = min(max(mc - 3 + i, 0), n_mc - 1)
            tm = m2 * n_sub + sb
            for c in range(8):
                k = min(max(ks - 3 + c, 0), K - 1)
                N = used[tm]
                ref = 0.0 if N == 0 else (stat[tm, k] / L - N) / np.sqrt(N)
                assert abs(f[region, 8 * i + c] - ref) <= 1e-5 * max(1.0, abs(ref))
