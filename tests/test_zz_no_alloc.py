"""The allocation-free PPO entry point (lob_ppo_fwd_bwd_noalloc) against the one that
takes a workspace (lob_ppo_fwd_bwd): two calls in a row through the C-ABI, the second
with a smaller minibatch, each bit-identical to the workspace entry point's result (same
kernels, same grid, same summation order) and both within the fused kernel's tolerance of
the float64 reference."""
import numpy as np
import pytest
import torch

from oracle import ppo_ref as R

pytestmark = pytest.mark.gpu


def _batch(rng, m, n_act, params):
    obs = rng.normal(0, 1, size=(m, 40)).astype(np.float32)
    logits, v = R.mlp_forward(params, obs)
    lp = R.log_softmax(logits, n_act)
    act = rng.integers(0, n_act, size=m)
    logp_old = lp[np.arange(m), act] + rng.normal(0, 0.05, size=m)
    adv = rng.normal(0, 1, size=m)
    ret = v + rng.normal(0, 0.5, size=m)
    v_old = v + rng.uniform(-0.1, 0.1, size=m)
    t = lambda x, d=torch.float32: torch.from_numpy(np.ascontiguousarray(x)).to("cuda", d)
    return (t(obs), t(act, torch.int32), t(logp_old.astype(np.float32)), t(adv.astype(np.float32)),
            t(ret.astype(np.float32)), t(v_old.astype(np.float32))), (obs, act, logp_old, adv, ret, v_old)


def test_noalloc_matches_the_workspace_entry_point():
    from paper_2511_02136_amd import ippo
    rng = np.random.default_rng(2024)
    params_np = R.xavier_init(rng)
    params = torch.from_numpy(params_np).cuda()
    loss_na = torch.empty(4, dtype=torch.float32, device="cuda")
    grad_na = torch.empty(ippo.N_PARAMS, dtype=torch.float32, device="cuda")
    for m in (131072, 200):
        print(f"\n[noalloc] m={m}", flush=True)
        dev, host = _batch(rng, m, 9, params_np)
        loss_w, grad_w = ippo.ppo_fwd_bwd(params, *dev, 9)
        ippo.ppo_fwd_bwd_noalloc(params, *dev, 9, loss_na, grad_na)
        torch.cuda.synchronize()
        assert torch.equal(loss_na, loss_w), m
        assert torch.equal(grad_na, grad_w), m
        if m <= 4096:
            ref_loss, ref_grad = R.ppo_loss_and_grad(params_np, *host, 9)
            g = grad_na.double().cpu().numpy()
            assert np.linalg.norm(g - ref_grad) <= 1e-5 * np.linalg.norm(ref_grad)
            assert abs(float(loss_na[0]) / m - ref_loss) <= 2e-5 * max(1.0, abs(ref_loss))
