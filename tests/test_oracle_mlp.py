"""The oracle's filter network equals torch.nn in FP64 (a library routine)."""
import numpy as np
import torch

from oracle import mlp
from synthetic import MLP_N_PARAMS, mlp_init, normal


def _torch_net(theta):
    net = torch.nn.Sequential(torch.nn.Linear(2, 64), torch.nn.SiLU(),
                              torch.nn.Linear(64, 64), torch.nn.SiLU(),
                              torch.nn.Linear(64, 1)).double()
    W1, b1, W2, b2, W3, b3 = mlp.unpack(theta)
    with torch.no_grad():
        for layer, (w, b) in zip((net[0], net[2], net[4]), ((W1, b1), (W2, b2), (W3, b3))):
            layer.weight.copy_(torch.from_numpy(w))
            layer.bias.copy_(torch.from_numpy(b))
    return net


def test_param_count():
    assert mlp.N_PARAMS == MLP_N_PARAMS == 4417


def test_forward_and_backward_match_torch():
    theta = mlp_init(3, zero_last=False)
    x = mlp.features(16, 32.0, 0.37)
    g, cache = mlp.forward(theta, x)
    net = _torch_net(theta)
    xt = torch.from_numpy(x)
    out = net(xt)[:, 0]
    np.testing.assert_allclose(g, out.detach().numpy(), rtol=1e-12, atol=1e-14)
    gbar = normal(x.shape[0], 4)
    out.backward(torch.from_numpy(gbar))
    ref = np.concatenate([p.grad.numpy().reshape(-1) for p in net.parameters()])
    np.testing.assert_allclose(mlp.backward(theta, cache, gbar), ref, rtol=1e-11, atol=1e-13)


def test_features_cover_every_integer_shell():
    x = mlp.features(8, 8.0, 0.5)
    assert x.shape == (3 * 16 + 1, 2)
    assert abs(x[-1, 0] - np.sqrt(3)) < 1e-15      # corner |k| = sqrt(3) k_Nyq
    assert np.all(x[:, 1] == 0.5)
