"""The allocation-free training step (tnmc_mlp_train_step_noalloc, static
per-GPU scratch) against the workspace form (tnmc_mlp_train_step) through
the C ABI: gradient, loss, Adam moments and parameters bit-identical, on two
calls in a row, the second with fewer rows (the static scratch then still
holds the first call's partials beyond the second call's range)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _rows(n, seed):
    rng = np.random.default_rng(seed)
    x = rng.normal(0, 1, (n, 64)).astype(np.float32)
    x[:, 53:] = 0
    lo = rng.normal(0, 3, n).astype(np.float32)
    tg = (lo + rng.normal(0, 0.7, n)).astype(np.float32)
    return x, lo, tg


def test_noalloc_train_step_equals_workspace_form(tnmc):
    import torch
    import tnmc_gpu as G
    rng = np.random.default_rng(3)
    P0 = torch.as_tensor(rng.uniform(-0.3, 0.3, tnmc.MLP_NPARAM).astype(np.float32)).cuda()
    state = {}
    for form in ("workspace", "noalloc"):
        P = P0.clone()
        m = torch.zeros_like(P)
        v = torch.zeros_like(P)
        outs = []
        for call, n in enumerate((5000, 777)):
            G.say(f"train step {form}, call {call}, {n} rows")
            x, lo, tg = (torch.as_tensor(a).cuda() for a in _rows(n, 10 + call))
            grad = torch.zeros(tnmc.MLP_NPARAM, dtype=torch.float32, device="cuda")
            loss = torch.zeros(1, dtype=torch.float32, device="cuda")
            if form == "workspace":
                scr = torch.zeros(tnmc.tnmc_mlp_scratch_floats(n), dtype=torch.float32, device="cuda")
                tnmc.tnmc_mlp_train_step(P, m, v, x, lo, tg, 1e-3, call + 1, scr, grad_out=grad, loss_out=loss)
            else:
                tnmc.tnmc_mlp_train_step_noalloc(P, m, v, x, lo, tg, 1e-3, call + 1, grad_out=grad, loss_out=loss)
            torch.cuda.synchronize()
            outs.append([t.cpu().numpy().copy() for t in (grad, loss, P, m, v)])
        state[form] = outs
    for call in range(2):
        for a, b in zip(state["workspace"][call], state["noalloc"][call]):
            assert np.array_equal(a, b), call
    # beyond the static limit: a clear error, nothing enqueued
    n = tnmc.MLP_NOALLOC_MAX_ROWS + 1
    x = torch.zeros((n, 64), dtype=torch.float32, device="cuda")
    lo = torch.zeros(n, dtype=torch.float32, device="cuda")
    with pytest.raises(tnmc.TnmcError) as e:
        tnmc.tnmc_mlp_train_step_noalloc(P0, None, None, x, lo, lo, 0.0, 0)
    assert e.value.code == tnmc.TNMC_EINVAL and "static scratch limit" in str(e.value)
