"""GPU training kernels of the learned proposal against the oracle.

Bars: the batch loss within 2e-3 relative of the oracle's BF16-emulating loss;
every entry of the gradient within the oracle's envelope of the device's
arithmetic (the BF16-emulating back-propagation with the device's rounding
points, plus the effect of every rounding that FP32 sums may take the other
way); the Adam step equals its formula applied to the reported gradient;
training lowers the loss on a learnable synthetic target.
"""
import math

import numpy as np
import pytest

import synth
from tests.gpu_helpers import flush

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]
HEAD = dict(m_max=1.0, lo=math.log(0.02), hi=math.log(1.0))
GROUPS = [("w1", 3840), ("b1", 64), ("w2", 4096), ("b2", 64), ("w3", 384), ("b3", 6)]


def _opts(C, apply, lr=1e-3, max_waves=0):
    return C.soma_train_opts(lr, 0.9, 0.999, 1e-8, HEAD["m_max"], HEAD["lo"], HEAD["hi"],
                             apply, max_waves)


def _step(C, params, f, t, apply=0, m=None, v=None, step=1, lr=1e-3, max_waves=0):
    n = f.shape[0]
    waves = (n + 63) // 64 if max_waves == 0 else min((n + 63) // 64, max_waves)
    ws = torch.empty(C.soma_train_workspace_bytes(waves), dtype=torch.uint8, device="cuda")
    grad = torch.empty(8576, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    C.soma_train_step(f.data_ptr(), t.data_ptr(), n, params.data_ptr(),
                      m.data_ptr() if m is not None else 0, v.data_ptr() if v is not None else 0,
                      step, _opts(C, apply, lr, max_waves), ws.data_ptr(), ws.numel(),
                      grad.data_ptr(), loss.data_ptr(), torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return grad.cpu().numpy().astype(np.float64), float(loss.item())


@pytest.mark.parametrize("n,max_waves", [(1000, 0), (4096, 7), (65, 0)])
def test_gradient_matches_bf16_oracle(orc, n, max_waves):
    """Every entry of the device's mean gradient lies within the oracle's
    envelope: the gradient with the device's rounding points (BF16 inputs,
    weights, activations and back-propagated errors) plus, per entry, the
    effect of every rounding that FP32 sums may take the other way, the FP32
    error bound of the unrounded bias terms and of the sums over samples."""
    from paper_1711_03828_amd import soma as C
    g = np.random.default_rng(n)
    params = synth.mlp_params(31, weight_gain=1.2, out_gain=0.5,
                              shift=g.standard_normal(60) * 0.1, scale=1 + 0.2 * g.random(60))
    f = (g.standard_normal((n, 60)) * 1.5).astype(np.float32)
    t = (g.standard_normal((n, 3)) * 0.3).astype(np.float32)
    p = torch.from_numpy(params).cuda()
    grad, loss = _step(C, p, torch.from_numpy(f).cuda(), torch.from_numpy(t).cuda(),
                       max_waves=max_waves)
    loss_o, grad_o, bound, n_amb, n_flag = orc.nll_batch_envelope(params, f, t, **HEAD)
    flush("loss", loss, loss_o, "ambiguous roundings", n_amb, "samples with one", n_flag)
    assert abs(loss - loss_o) <= 2e-3 * abs(loss_o)
    L = synth.MLP_LAYOUT
    for name, size in GROUPS:
        sl = slice(L[name], L[name] + size)
        d = np.abs(grad[sl] - grad_o[sl])
        rms = np.sqrt(np.mean(grad_o[sl] ** 2))
        flush(name, "max |dg|/rms", d.max() / rms, "median bound/rms", np.median(bound[sl]) / rms,
              "max |dg|/bound", (d / np.maximum(bound[sl], 1e-300)).max())
        assert (d <= bound[sl]).all(), (name, int(np.argmax(d - bound[sl])))
    assert np.all(grad[:120] == 0.0) and np.all(grad[8574:] == 0.0)


def test_adam_step_formula():
    from paper_1711_03828_amd import soma as C
    g = np.random.default_rng(3)
    params = synth.mlp_params(32)
    f = torch.from_numpy((g.standard_normal((512, 60))).astype(np.float32)).cuda()
    t = torch.from_numpy((g.standard_normal((512, 3)) * 0.3).astype(np.float32)).cuda()
    p = torch.from_numpy(params.copy()).cuda()
    m = torch.zeros(8576, device="cuda")
    v = torch.zeros(8576, device="cuda")
    grad, _ = _step(C, p, f, t, apply=1, m=m, v=v, step=1, lr=1e-2)
    new = p.cpu().numpy().astype(np.float64)
    gr = grad
    mm = 0.1 * gr
    vv = 0.001 * gr * gr
    exp = params.astype(np.float64) - 1e-2 * (mm / 0.1) / (np.sqrt(vv / 0.001) + 1e-8)
    trainable = np.zeros(8576, bool)
    trainable[120:8574] = True
    np.testing.assert_allclose(new[trainable], exp[trainable], rtol=1e-5, atol=1e-6)
    np.testing.assert_array_equal(new[~trainable], params[~trainable])


def test_training_reduces_loss():
    from paper_1711_03828_amd import learned
    g = np.random.default_rng(4)
    n = 20000
    f = g.standard_normal((n, 60)).astype(np.float32)
    # displacement: 0.3 x the previous bond vector plus noise of std 0.1
    t = (0.3 * f[:, 54:57] + 0.1 * g.standard_normal((n, 3))).astype(np.float32)
    ft = torch.from_numpy(f).cuda()
    tt = torch.from_numpy(t).cuda()
    params = learned.init_params(ft, seed=1)
    losses = learned.train(params, ft, tt, steps=300, batch=2048, lr=3e-3)
    flush("loss start", losses[0], "end", np.mean(losses[-20:]))
    # the optimum: log-likelihood of N(0.3 f, 0.1^2): sum_d log 0.1 + 1/2 = -5.41
    assert np.mean(losses[-20:]) < losses[0] - 2.0
    assert np.mean(losses[-20:]) < -4.0
