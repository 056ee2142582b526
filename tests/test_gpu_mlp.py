"""GPU parity of the warm-start network kernels (pbs_mlp_*) against the
oracle: forward pass, loss and every gradient block, and an Adam trajectory,
at the 1 -> 256 -> 256 -> 200 shape and at ragged shapes that exercise the
batch and output padding.

Tolerances.  Both sides multiply the same bf16-rounded weights; the kernel
accumulates in float32 (error <= K u32 sum|a b|, about 1.5e-5 relative for
K = 256), and rounds its own float32 activations to bf16 where the oracle
rounds float64 ones.  The two roundings differ by one bf16 ulp (2^-8
relative) only for operands whose float32 and float64 values straddle a
rounding boundary: a fraction of about K u32 / 2^-8 (~2e-3) of them, each
moving a K-term sum by 2^-8 / sqrt(K) in the relative 2-norm, so the
expected effect is ~1e-5 and BOUND = 2^-12 (2.4e-4) holds outputs, losses
and gradient blocks with room to spare, while a wrong index, operand or
rounding point shows up at 1e-2 or more."""

import numpy as np
import pytest
import torch

import synth
from oracle import mlp as omlp

pytestmark = pytest.mark.gpu

BOUND = 2.0 ** -12


def _api():
    from paper_2606_28952_amd import api

    return api


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def _blocks(v, H, O):
    return dict(zip(["W1", "b1", "W2", "b2", "W3", "b3"], omlp.unpack(v, H, O)))


def _data(n, O, seed):
    rng = np.random.default_rng(seed)
    x = np.sort(rng.uniform(0, 1, n)).astype(np.float32)
    basis = np.stack([np.sin((k % 7 + 1) * x + k) * (0.2 + 0.01 * (k % 5)) for k in range(O)], axis=1)
    return x, basis.astype(np.float32)


SHAPES = [(256, 200, 40), (256, 200, 1), (64, 5, 3), (32, 33, 33), (96, 64, 70)]


@pytest.mark.parametrize("H,O,n", SHAPES)
def test_forward_matches_oracle(dev, H, O, n):
    api = _api()
    p = synth.mlp_init(H, O, seed=H + O + n)
    x, _ = _data(n, O, seed=n)
    net = api.MLP(H, O, max(n, 8), p)
    y = net.forward(torch.from_numpy(x).to(dev)).cpu().numpy()
    want, _ = omlp.forward(p.astype(np.float64), x.astype(np.float64), H, O)
    assert y.shape == (n, O)
    assert _rel(y, want) < BOUND


@pytest.mark.parametrize("H,O,n", SHAPES)
def test_loss_and_gradients_match_oracle(dev, H, O, n):
    api = _api()
    p = synth.mlp_init(H, O, seed=3 * H + O)
    x, t = _data(n, O, seed=n + 1)
    net = api.MLP(H, O, n, p)
    loss, g = net.loss_grad(torch.from_numpy(x).to(dev), torch.from_numpy(t).to(dev))
    want_l, want_g = omlp.loss_grad(p.astype(np.float64), x.astype(np.float64), t.astype(np.float64), H, O)
    assert abs(loss.item() - want_l) < BOUND * want_l
    got = _blocks(g.cpu().numpy(), H, O)
    for name, ref in _blocks(want_g, H, O).items():
        assert _rel(got[name], ref) < BOUND, name
    # the parameters are untouched by a gradient evaluation
    np.testing.assert_array_equal(net.params(), p)


def test_adam_trajectory_matches_oracle(dev):
    api = _api()
    H, O, n, steps, lr = 256, 200, 24, 30, 1e-3
    p = synth.mlp_init(H, O, seed=12)
    x, t = _data(n, O, seed=5)
    net = api.MLP(H, O, 64, p)
    losses = net.train(torch.from_numpy(x).to(dev), torch.from_numpy(t).to(dev), steps, lr).cpu().numpy()
    q, want_losses, _ = omlp.train(p.astype(np.float64), x, t, H, O, steps, lr)
    assert np.all(np.abs(losses - want_losses) < 16 * BOUND * want_losses)
    assert losses[-1] < 0.5 * losses[0]
    got = net.params().astype(np.float64)
    # Adam divides by the root of the second moment, which amplifies the
    # gradient differences of weights whose gradients are near zero; the
    # moves still agree to a few percent of the bf16 step
    assert _rel(got - p, q - p) < 64 * BOUND


def test_training_generalises_between_samples(dev):
    api = _api()
    H, O = 256, 200
    x, t = _data(32, O, seed=9)
    train_idx = np.arange(0, 32, 2)
    test_idx = np.arange(1, 31, 2)
    net = api.MLP(H, O, 64, synth.mlp_init(H, O, seed=1))
    xs = torch.from_numpy(x[train_idx]).to(dev)
    ts = torch.from_numpy(t[train_idx]).to(dev)
    net.train(xs, ts, 1500, 2e-3)
    pred = net.forward(torch.from_numpy(x[test_idx]).to(dev)).cpu().numpy()
    err = np.sqrt(np.mean((pred - t[test_idx]) ** 2))
    base = np.sqrt(np.mean(t[test_idx] ** 2))
    assert err < 0.05 * base


def test_argument_errors(dev):
    api = _api()
    p = synth.mlp_init(32, 4, seed=0)
    with pytest.raises(ValueError):
        api.MLP(32, 5, 8, p)
    with pytest.raises(Exception, match="hidden"):
        api.MLP(48, 4, 8, synth.mlp_init(48, 4, seed=0))
    net = api.MLP(32, 4, 8, p)
    with pytest.raises(Exception, match="batch"):
        net.forward(torch.zeros(9, device=dev))


def test_training_runs_match_single_steps(dev):
    # the Adam step count lives on the device: one call of n steps and n
    # calls of one step, with forward passes between the runs, give
    # bit-identical parameters and losses
    api = _api()
    H, O, n = 64, 20, 12
    p = synth.mlp_init(H, O, seed=21)
    x, t = _data(n, O, seed=22)
    xs, ts = torch.from_numpy(x).to(dev), torch.from_numpy(t).to(dev)
    run_net, eager_net = api.MLP(H, O, n, p), api.MLP(H, O, n, p)
    run_losses, eager_losses = [], []
    for run in (20, 9):
        run_losses.append(run_net.train(xs, ts, run, 2e-3).cpu().numpy())
        run_net.forward(xs)
        for _ in range(run):
            eager_losses.append(eager_net.train(xs, ts, 1, 2e-3).cpu().numpy())
        eager_net.forward(xs)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(run_net.params(), eager_net.params())
    np.testing.assert_array_equal(np.concatenate(run_losses), np.concatenate(eager_losses))
    assert not np.array_equal(run_net.params(), p)


def test_captured_training_replays_continue_the_count(dev):
    """A training call captured in a HIP graph and replayed several times,
    then called directly: every replay and call writes its losses into slots
    0..n_steps-1 of its own buffer (nothing past them), and parameters and
    losses equal those of the same calls made directly, bit for bit."""
    api = _api()
    H, O, n, k = 64, 20, 12, 3
    p = synth.mlp_init(H, O, seed=31)
    x, t = _data(n, O, seed=32)
    xs, ts = torch.from_numpy(x).to(dev), torch.from_numpy(t).to(dev)
    cap_net, eager_net = api.MLP(H, O, n, p), api.MLP(H, O, n, p)
    guard = 5
    buf = torch.full((k + guard,), float("nan"), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        with torch.cuda.graph(graph, stream=stream):
            cap_net.train_into(xs, ts, k, 2e-3, buf)
    torch.cuda.synchronize()
    for rep in range(3):
        buf.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        want = eager_net.train(xs, ts, k, 2e-3).cpu().numpy()
        got = buf.cpu().numpy()
        np.testing.assert_array_equal(got[:k], want, err_msg=f"replay {rep}")
        assert np.isnan(got[k:]).all(), f"replay {rep} wrote past its losses"
    direct = torch.full((2 + guard,), float("nan"), dtype=torch.float32, device=dev)
    cap_net.train_into(xs, ts, 2, 2e-3, direct)
    want = eager_net.train(xs, ts, 2, 2e-3).cpu().numpy()
    got = direct.cpu().numpy()
    np.testing.assert_array_equal(got[:2], want)
    assert np.isnan(got[2:]).all()
    np.testing.assert_array_equal(cap_net.params(), eager_net.params())
