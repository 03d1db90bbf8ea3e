"""GPU parity of the actor-critic kernels (policy forward, sampling, GAE, fused PPO).

Floating-point tolerances (fp32 kernels vs the float64 oracle): forward outputs and loss
sums within 2e-5 relative to their scale (fp32 accumulation over 256-term dot products);
the PPO gradient within 1e-5 relative (norm-wise) of both the float64 autograd gradient
and float64 central finite differences on sampled coordinates; GAE within 1e-5.
Sampled actions (an argmax decided in float) are checked for consistency with the
float64 decision wherever the margin exceeds 1e-3, and for their distribution.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import ppo_ref as R
from test_ppo_ref import batch

pytestmark = pytest.mark.gpu

DOM_POLICY = 0x504F4C4943


def _ippo():
    from paper_2511_02136_amd import ippo
    return ippo


def rand_params(seed, n_agents=1):
    rng = np.random.default_rng(seed)
    ps = []
    for _ in range(n_agents):
        p = R.xavier_init(rng)
        for k in ("b1", "b2", "b3"):
            a, b, _ = R.SLICES[k]
            p[a:b] = rng.normal(0, 0.1, b - a).astype(np.float32)
        ps.append(p)
    return np.stack(ps)


def test_policy_forward_matches_fp64_and_samples_consistently():
    ippo = _ippo()
    A, n = 2, 200
    P = rand_params(1, A)
    rng = np.random.default_rng(2)
    obs = rng.normal(0, 1, size=(A, n, 40)).astype(np.float32)
    n_act = [9, 3]
    out = ippo.policy_forward(torch.from_numpy(P).cuda(), torch.from_numpy(obs).cuda(), n_act, seed=7, t=3,
                              want_logits=True)
    torch.cuda.synchronize()
    lg = out["logits"].cpu().numpy().astype(np.float64)
    for ag in range(A):
        ref_l, ref_v = R.mlp_forward(P[ag], obs[ag])
        scale = np.abs(ref_l).max() + 1
        assert np.abs(lg[ag, :, :9] - ref_l).max() <= 2e-5 * scale
        assert np.abs(out["value"][ag].cpu().numpy() - ref_v).max() <= 2e-5 * (np.abs(ref_v).max() + 1)
        # sampling: Gumbel-max with the counter-hash noise, recomputed in float64
        z = lg[ag, :, :n_act[ag]]
        acts = out["actions"][ag].cpu().numpy()
        checked = 0
        for e in range(n):
            u = np.array([((oracle.chain_hash(7, DOM_POLICY, (ag << 8) | j, 3, e) >> 40) + 0.5) / 16777216.0
                          for j in range(n_act[ag])])
            s = z[e] - np.log(-np.log(u))
            order = np.argsort(-s)
            if s[order[0]] - s[order[1]] > 1e-3:
                assert acts[e] == order[0], (ag, e)
                checked += 1
        assert checked > 0.9 * n
        lse = z.max(1) + np.log(np.exp(z - z.max(1, keepdims=True)).sum(1))
        ref_lp = z[np.arange(n), acts] - lse
        assert np.abs(out["logp"][ag].cpu().numpy() - ref_lp).max() <= 2e-5


def test_sampling_distribution():
    ippo = _ippo()
    n = 4000
    P = np.zeros((1, R.N_PARAMS), dtype=np.float32)
    a, b, _ = R.SLICES["b3"]
    target = np.array([0.0, 1.0, -1.0, 0.5, 2.0, 0, 0, 0, 0], dtype=np.float32)
    P[0, a:a + 9] = target
    obs = torch.zeros((1, n, 40), dtype=torch.float32, device="cuda")
    counts = np.zeros(5)
    for t in range(5):
        out = ippo.policy_forward(torch.from_numpy(P).cuda(), obs, [5], seed=11, t=t)
        counts += np.bincount(out["actions"][0].cpu().numpy(), minlength=5)
    p = np.exp(target[:5]) / np.exp(target[:5]).sum()
    expect = counts.sum() * p
    chi2 = ((counts - expect) ** 2 / expect).sum()
    assert chi2 < 25.0  # 4 dof


def test_gae_matches_fp64():
    ippo = _ippo()
    rng = np.random.default_rng(5)
    T, n = 128, 777
    r = rng.normal(size=(T, n)).astype(np.float32)
    v = rng.normal(size=(T, n)).astype(np.float32)
    d = np.zeros((T, n), dtype=np.uint8)
    d[-1] = 1
    d[60, ::3] = 1
    last = rng.normal(size=n).astype(np.float32)
    adv, ret = ippo.gae(*(torch.from_numpy(x).cuda() for x in (r, v, d, last)), gamma=0.99, lam=0.95)
    ra, rr = R.gae(r, v, d, last, 0.99, 0.95)
    assert np.abs(adv.cpu().numpy() - ra).max() <= 1e-5 * (np.abs(ra).max() + 1)
    assert np.abs(ret.cpu().numpy() - rr).max() <= 1e-5 * (np.abs(rr).max() + 1)


# 16,401 samples: more 64-sample tiles (257) than the kernel's 256 workgroups, the last
# tile ragged and summed by workgroup 0 after its first; 1 sample: one ragged tile
@pytest.mark.parametrize("m,n_act,big", [(200, 9, False), (130, 3, True), (64, 9, True), (1, 9, False),
                                         (16401, 5, False)])
def test_fused_ppo_loss_and_gradient(m, n_act, big):
    ippo = _ippo()
    rng = np.random.default_rng(m + n_act)
    P = rand_params(m, 1)[0]
    P64 = P.astype(np.float64)
    obs, act, lpo, adv, ret, vo = batch(rng, m, n_act, P64, big=big)
    dev = [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in (P, obs, act.astype(np.int32), lpo, adv, ret, vo)]
    loss, grad = ippo.ppo_fwd_bwd(*dev, n_act)
    torch.cuda.synchronize()
    loss, grad = loss.cpu().numpy().astype(np.float64), grad.cpu().numpy().astype(np.float64)
    tot, pol, val, ent = R.ppo_loss_parts(P64, obs, act, lpo, adv, ret, vo, n_act)
    for got, ref in zip(loss / m, (tot, pol, val, ent)):
        assert abs(got - ref) <= 2e-5 * (abs(ref) + 1e-3)
    ref_loss, ref_grad = R.ppo_loss_and_grad(P64, obs, act, lpo, adv, ret, vo, n_act)
    err = np.linalg.norm(grad - ref_grad) / np.linalg.norm(ref_grad)
    assert err <= 1e-5, err
    # central finite differences of the float64 loss on sampled coordinates of every tensor
    idx = np.concatenate([rng.choice(np.arange(a, b), size=min(20, b - a), replace=False)
                          for a, b, _ in R.SLICES.values()])
    h = 1e-6
    fd = np.empty(len(idx))
    for j, i in enumerate(idx):
        pp = P64.copy(); pp[i] += h
        pm = P64.copy(); pm[i] -= h
        fd[j] = (R.ppo_loss_parts(pp, obs, act, lpo, adv, ret, vo, n_act)[0] -
                 R.ppo_loss_parts(pm, obs, act, lpo, adv, ret, vo, n_act)[0]) / (2 * h)
    err_fd = np.linalg.norm(grad[idx] - fd) / np.linalg.norm(fd)
    assert err_fd <= 1e-5, err_fd
    # deterministic
    _, grad2 = ippo.ppo_fwd_bwd(*dev, n_act)
    assert np.array_equal(grad2.cpu().numpy().astype(np.float64), grad)


def test_fused_ppo_with_unaligned_parameters():
    """The second network of a [2][78858] array starts 315,432 bytes in (not a multiple of
    16): the call copies it to aligned workspace first and must give the same loss and
    gradient, bit for bit, as the same values in their own allocation."""
    ippo = _ippo()
    rng = np.random.default_rng(21)
    P2 = rand_params(21, 2)
    obs, act, lpo, adv, ret, vo = batch(rng, 150, 9, P2[1].astype(np.float64))
    args = [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in (obs, act.astype(np.int32), lpo, adv, ret, vo)]
    both = torch.from_numpy(P2).cuda()
    row = both[1]
    assert row.data_ptr() % 16 != 0
    loss_a, grad_a = ippo.ppo_fwd_bwd(row, *args, 9)
    loss_b, grad_b = ippo.ppo_fwd_bwd(row.clone(), *args, 9)
    assert torch.equal(loss_a, loss_b) and torch.equal(grad_a, grad_b)
    assert torch.equal(both[1], torch.from_numpy(P2[1]).cuda())  # the input is not modified
    ref_loss, ref_grad = R.ppo_loss_and_grad(P2[1].astype(np.float64), obs, act, lpo, adv, ret, vo, 9)
    err = np.linalg.norm(grad_a.cpu().numpy().astype(np.float64) - ref_grad) / np.linalg.norm(ref_grad)
    assert err <= 1e-5, err


def test_autograd_function_and_optimizer_step():
    ippo = _ippo()
    rng = np.random.default_rng(9)
    P = rand_params(9, 1)[0]
    obs, act, lpo, adv, ret, vo = batch(rng, 96, 9, P.astype(np.float64))
    params = torch.nn.Parameter(torch.from_numpy(P).cuda())
    args = [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in (obs, act.astype(np.int32), lpo, adv, ret, vo)]
    loss = ippo.FusedPPOLoss.apply(params, *args, 9)
    loss.backward()
    _, grad = ippo.ppo_fwd_bwd(params.detach(), *args, 9)
    assert torch.equal(params.grad, grad)
    opt = torch.optim.Adam([params], lr=1e-3)
    before = params.detach().clone()
    opt.step()
    assert not torch.equal(before, params.detach())
    loss2 = ippo.FusedPPOLoss.apply(params, *args, 9)
    assert float(loss2) < float(loss)  # one small step along -grad lowers the loss


@pytest.mark.parametrize("m", [131072, 1048576])
def test_full_size_minibatch_gradient(m):
    """Full-size minibatches in the launch configuration of the update: ippo4096 (4096 envs
    x 128 steps / 4 = 131072 samples) and the large workload (16384 envs x 256 steps / 4 =
    1048576 samples), against float64 autograd on the CPU."""
    ippo = _ippo()
    print(f"\n[ppo] minibatch of {m} samples", flush=True)
    rng = np.random.default_rng(12)
    P = rand_params(12, 1)[0]
    P64 = P.astype(np.float64)
    obs = rng.normal(0, 1, size=(m, 40)).astype(np.float32)
    act = rng.integers(0, 9, size=m)
    logits, v = R.mlp_forward(P64, obs)
    lp = R.log_softmax(logits, 9)
    lpo = (lp[np.arange(m), act] + rng.normal(0, 0.05, size=m)).astype(np.float32)
    adv = rng.normal(size=m).astype(np.float32)
    ret = (v + rng.normal(0, 0.5, size=m)).astype(np.float32)
    vo = (v + rng.uniform(-0.15, 0.15, size=m)).astype(np.float32)
    dev = [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in (P, obs, act.astype(np.int32), lpo, adv, ret, vo)]
    loss, grad = ippo.ppo_fwd_bwd(*dev, 9)
    torch.cuda.synchronize()
    ref_loss, ref_grad = R.ppo_loss_and_grad(P64, obs, act, lpo, adv, ret, vo, 9)
    assert abs(float(loss[0]) / m - ref_loss) <= 2e-5 * (abs(ref_loss) + 1e-3)
    err = np.linalg.norm(grad.cpu().numpy().astype(np.float64) - ref_grad) / np.linalg.norm(ref_grad)
    assert err <= 1e-5, err


def test_observation_scale_inside_the_kernels():
    """The policy's input scaling given to the kernels equals scaling the observations
    first: policy forward bit for bit (the kernel multiplies as torch does), the PPO loss
    and gradient bit for bit."""
    ippo = _ippo()
    rng = np.random.default_rng(41)
    P = torch.from_numpy(rand_params(41, 2)).cuda()
    obs = torch.from_numpy(rng.normal(0, 50, size=(2, 96, 40)).astype(np.float32)).cuda()
    sc = torch.from_numpy(rng.uniform(0.001, 0.5, size=40).astype(np.float32)).cuda()
    a = ippo.policy_forward(P, obs, [9, 3], seed=3, t=1, want_logits=True, obs_scale=sc)
    b = ippo.policy_forward(P, (obs * sc).contiguous(), [9, 3], seed=3, t=1, want_logits=True)
    for k in ("actions", "logp", "value", "logits"):
        assert torch.equal(a[k], b[k]), k
    m = 130
    o = obs[0, :96].contiguous()
    o = torch.cat([o, o[:34]]).contiguous()
    act = torch.from_numpy(rng.integers(0, 9, size=m).astype(np.int32)).cuda()
    lpo, adv, ret, vo = (torch.from_numpy(rng.normal(0, 1, size=m).astype(np.float32)).cuda() for _ in range(4))
    la, ga = ippo.ppo_fwd_bwd(P[0].contiguous(), o, act, lpo, adv, ret, vo, 9, obs_scale=sc)
    lb, gb = ippo.ppo_fwd_bwd(P[0].contiguous(), (o * sc).contiguous(), act, lpo, adv, ret, vo, 9)
    assert torch.equal(la, lb) and torch.equal(ga, gb)
