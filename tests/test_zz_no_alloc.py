"""soma_train_step_noalloc (the training step without a workspace argument:
its scratch is a fixed device array of the library) against soma_train_step.

Both run the same kernels with the same number of partial gradients, so the
gradient, the loss and the Adam update must be bit-identical.  Two calls in a
row, the second with a smaller batch (the array keeps the first call's
contents); each call is also checked against the workspace entry point on the
same inputs.  Sizes beyond the array are refused with SOMA_E_SIZE.
"""
import math

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def _opts(C, apply, max_waves):
    return C.soma_train_opts(1e-3, 0.9, 0.999, 1e-8, 1.0, math.log(0.02), math.log(1.0),
                             apply, max_waves)


def _run(C, noalloc, params, m, v, f, t, step, max_waves):
    n = f.shape[0]
    grad = torch.full((8576,), float("nan"), dtype=torch.float32, device="cuda")
    loss = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    opts = _opts(C, 1, max_waves)
    if noalloc:
        C.soma_train_step_noalloc(f.data_ptr(), t.data_ptr(), n, params.data_ptr(), m.data_ptr(),
                                  v.data_ptr(), step, opts, grad.data_ptr(), loss.data_ptr(),
                                  stream)
    else:
        chunks = (n + 63) // 64
        waves = chunks if max_waves == 0 else min(chunks, max_waves)
        ws = torch.empty(C.soma_train_workspace_bytes(waves), dtype=torch.uint8, device="cuda")
        C.soma_train_step(f.data_ptr(), t.data_ptr(), n, params.data_ptr(), m.data_ptr(),
                          v.data_ptr(), step, opts, ws.data_ptr(), ws.numel(), grad.data_ptr(),
                          loss.data_ptr(), stream)
    torch.cuda.synchronize()
    return grad.cpu().numpy(), loss.cpu().numpy()


def test_noalloc_train_step_equals_workspace_entry_point():
    from paper_1711_03828_amd import soma as C
    g = np.random.default_rng(17)
    base = synth.mlp_params(41, weight_gain=1.1, out_gain=0.4)
    state = {}
    for noalloc in (False, True):
        state[noalloc] = [torch.from_numpy(base.copy()).cuda(),
                          torch.zeros(8576, dtype=torch.float32, device="cuda"),
                          torch.zeros(8576, dtype=torch.float32, device="cuda")]
    # second call smaller than the first: 5000 samples on 40 partials, then 300
    # samples on one partial per 64 samples
    for step, (n, max_waves) in enumerate([(5000, 40), (300, 0)], start=1):
        f = torch.from_numpy((g.standard_normal((n, 60)) * 1.3).astype(np.float32)).cuda()
        t = torch.from_numpy((g.standard_normal((n, 3)) * 0.3).astype(np.float32)).cuda()
        out = {}
        for noalloc in (False, True):
            p, m, v = state[noalloc]
            out[noalloc] = _run(C, noalloc, p, m, v, f, t, step, max_waves)
        assert np.isfinite(out[True][0]).all() and np.isfinite(out[True][1]).all()
        np.testing.assert_array_equal(out[True][0], out[False][0], err_msg=f"gradient, call {step}")
        np.testing.assert_array_equal(out[True][1], out[False][1], err_msg=f"loss, call {step}")
        for k in range(3):
            assert torch.equal(state[True][k], state[False][k]), (step, k)


def test_noalloc_train_step_refuses_oversized_batches():
    from paper_1711_03828_amd import soma as C
    n = 64 * (C.SOMA_NOALLOC_TRAIN_WAVES + 1)
    f = torch.zeros((n, 60), dtype=torch.float32, device="cuda")
    t = torch.zeros((n, 3), dtype=torch.float32, device="cuda")
    p = torch.from_numpy(synth.mlp_params(1)).cuda()
    m = torch.zeros(8576, dtype=torch.float32, device="cuda")
    v = torch.zeros(8576, dtype=torch.float32, device="cuda")
    with pytest.raises(C.SomaError, match="partial") as err:
        C.soma_train_step_noalloc(f.data_ptr(), t.data_ptr(), n, p.data_ptr(), m.data_ptr(),
                                  v.data_ptr(), 1, _opts(C, 1, 0), 0, 0,
                                  torch.cuda.current_stream().cuda_stream)
    assert err.value.code == C.SOMA_E_SIZE
    # the same batch on at most SOMA_NOALLOC_TRAIN_WAVES partials is accepted
    grad = torch.empty(8576, dtype=torch.float32, device="cuda")
    C.soma_train_step_noalloc(f.data_ptr(), t.data_ptr(), n, p.data_ptr(), m.data_ptr(),
                              v.data_ptr(), 1, _opts(C, 0, C.SOMA_NOALLOC_TRAIN_WAVES),
                              grad.data_ptr(), 0, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert torch.isfinite(grad).all()
