"""IPPO actor-critic on the GPU: policy forward with sampling, GAE, and the fused
clipped-PPO loss with its hand-written backward behind ``torch.autograd.Function``.

Argument marshalling only; the computation runs in ``liblob.so`` (MFMA kernels).
Each agent type has its own network (independent PPO, Sec. 4.2 of the paper).
"""
from __future__ import annotations

import ctypes
from typing import Sequence

import numpy as np
import torch

from .lob import lib, _check, _p, _stream, LobError

N_PARAMS = 78858
GRU_PARAMS = 105610
GRU_HIDDEN = 128
OBS_DIM = 40

_ready = False


def _lib():
    global _ready
    L = lib()
    if not _ready:
        p, i32, i64, f32, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_uint64
        L.lob_policy_forward.argtypes = [p, p, p, i32, i32, p, u64, p, i32, p, p, p, p, p]
        L.lob_counter_bump.argtypes = [p, p]
        L.lob_counter_bump.restype = ctypes.c_int
        L.lob_policy_forward.restype = ctypes.c_int
        L.lob_gae.argtypes = [p, p, p, p, i32, i32, f32, f32, p, p, p]
        L.lob_gae.restype = ctypes.c_int
        L.lob_ppo_workspace_bytes.argtypes = [i32]
        L.lob_ppo_workspace_bytes.restype = i64
        L.lob_ppo_fwd_bwd.argtypes = [p, p, p, p, p, p, p, p, i32, i32, f32, f32, f32, p, i64, p, p, p]
        L.lob_ppo_fwd_bwd.restype = ctypes.c_int
        L.lob_ppo_fwd_bwd_noalloc.argtypes = [p, p, p, p, p, p, p, p, i32, i32, f32, f32, f32, p, p, p]
        L.lob_ppo_fwd_bwd_noalloc.restype = ctypes.c_int
        L.lob_gru_step.argtypes = [p, p, p, p, p, p, i32, i32, p, u64, p, i32, p, p, p, p, p]
        L.lob_gru_step.restype = ctypes.c_int
        L.lob_gru_ppo_workspace_bytes.argtypes = [i32, i32]
        L.lob_gru_ppo_workspace_bytes.restype = i64
        L.lob_gru_ppo_fwd_bwd.argtypes = [p, p, p, p, p, p, p, p, p, p, i32, i32, i32, f32, f32, f32, p, i64, p, p, p]
        L.lob_gru_ppo_fwd_bwd.restype = ctypes.c_int
        _ready = True
    return L


def _f32(t: torch.Tensor) -> torch.Tensor:
    if t.dtype != torch.float32 or not t.is_contiguous():
        raise LobError("expected a contiguous float32 tensor")
    return t


def xavier_params(n_agents: int, seed: int, device="cuda") -> torch.Tensor:
    """Glorot-uniform weights and zero biases for n_agents networks, [n_agents, N_PARAMS]."""
    g = torch.Generator().manual_seed(seed)
    out = torch.zeros(n_agents, N_PARAMS, dtype=torch.float32)
    shapes = ((40, 256), (256,), (256, 256), (256,), (256, 10), (10,))
    for a in range(n_agents):
        o = 0
        for s in shapes:
            n = int(np.prod(s))
            if len(s) == 2:
                lim = float(np.sqrt(6.0 / (s[0] + s[1])))
                out[a, o:o + n] = (torch.rand(n, generator=g) * 2 - 1) * lim
            o += n
    return out.to(device)


def counter_bump(counter: torch.Tensor):
    """counter += 1 on the device (graph-capturable); counter: uint64/int64 [1]."""
    _check(_lib().lob_counter_bump(_p(counter), _stream()), "lob_counter_bump")


def _scale(obs_scale):
    return None if obs_scale is None else _f32(obs_scale)


def policy_forward(params: torch.Tensor, obs: torch.Tensor, n_actions: Sequence[int], seed: int, t: int,
                   want_logits: bool = False, epoch: torch.Tensor = None, out: dict = None,
                   obs_scale: torch.Tensor = None) -> dict:
    """params [A, N_PARAMS], obs [A, n, 40] (float32, device; scaled by obs_scale [40]
    in the kernel when given) -> actions, logp, value [A, n]."""
    A, n = obs.shape[0], obs.shape[1]
    dev = obs.device
    if out is None:
        out = {"actions": torch.empty((A, n), dtype=torch.int32, device=dev),
               "logp": torch.empty((A, n), dtype=torch.float32, device=dev),
               "value": torch.empty((A, n), dtype=torch.float32, device=dev),
               "logits": torch.empty((A, n, 10), dtype=torch.float32, device=dev) if want_logits else None}
    na = (ctypes.c_int32 * A)(*[int(x) for x in n_actions])
    _check(_lib().lob_policy_forward(_p(_f32(params)), _p(_f32(obs)), _p(_scale(obs_scale)), A, n, na, seed,
                                     _p(epoch), t,
                                     _p(out.get("logits")), _p(out["actions"]), _p(out["logp"]), _p(out["value"]),
                                     _stream()), "lob_policy_forward")
    return out


def gae(rewards: torch.Tensor, values: torch.Tensor, dones: torch.Tensor, last_value: torch.Tensor,
        gamma: float = 0.99, lam: float = 0.95):
    """rewards, values [T, n] float32, dones [T, n] uint8, last_value [n] -> (adv, ret)."""
    T, n = rewards.shape
    adv = torch.empty_like(rewards)
    ret = torch.empty_like(rewards)
    d = dones.to(torch.uint8).contiguous()
    _check(_lib().lob_gae(_p(_f32(rewards)), _p(_f32(values)), _p(d), _p(_f32(last_value)), T, n, gamma, lam,
                          _p(adv), _p(ret), _stream()), "lob_gae")
    return adv, ret


def workspace_bytes(m: int) -> int:
    """Device workspace the fused PPO kernel needs for a minibatch of m samples."""
    return int(_lib().lob_ppo_workspace_bytes(int(m)))


def ppo_fwd_bwd(params, obs, act, logp_old, adv, ret, v_old, n_actions, clip=0.2, c_v=0.5, c_e=0.01,
                workspace=None, obs_scale=None):
    """Loss sums [4] (total, policy, value, entropy) and the gradient of the mean loss."""
    m = obs.shape[0]
    L = _lib()
    need = int(L.lob_ppo_workspace_bytes(m))
    if workspace is None or workspace.numel() * 4 < need:
        workspace = torch.empty((need + 3) // 4, dtype=torch.float32, device=obs.device)
    loss = torch.empty(4, dtype=torch.float32, device=obs.device)
    grad = torch.empty(N_PARAMS, dtype=torch.float32, device=obs.device)
    _check(L.lob_ppo_fwd_bwd(_p(_f32(params)), _p(_f32(obs)), _p(_scale(obs_scale)),
                             _p(act.to(torch.int32).contiguous()),
                             _p(_f32(logp_old)), _p(_f32(adv)), _p(_f32(ret)), _p(_f32(v_old)), m, int(n_actions),
                             clip, c_v, c_e, _p(workspace), workspace.numel() * 4, _p(loss), _p(grad), _stream()),
           "lob_ppo_fwd_bwd")
    return loss, grad


def ppo_fwd_bwd_noalloc(params, obs, act, logp_old, adv, ret, v_old, n_actions, loss, grad, clip=0.2, c_v=0.5,
                        c_e=0.01, obs_scale=None):
    """As ppo_fwd_bwd into caller-given loss [4] and grad [N_PARAMS] (float32, device),
    with the library's fixed scratch instead of a workspace: the call allocates nothing."""
    m = obs.shape[0]
    _check(_lib().lob_ppo_fwd_bwd_noalloc(_p(_f32(params)), _p(_f32(obs)), _p(_scale(obs_scale)), _p(act),
                                          _p(_f32(logp_old)),
                                          _p(_f32(adv)), _p(_f32(ret)), _p(_f32(v_old)), m, int(n_actions), clip, c_v,
                                          c_e, _p(_f32(loss)), _p(_f32(grad)), _stream()),
           "lob_ppo_fwd_bwd_noalloc")
    return loss, grad


def gru_init_params(n_agents: int, seed: int, device="cuda") -> torch.Tensor:
    """Glorot-uniform matrices and zero biases for n_agents recurrent networks,
    [n_agents, GRU_PARAMS]."""
    g = torch.Generator().manual_seed(seed)
    out = torch.zeros(n_agents, GRU_PARAMS, dtype=torch.float32)
    shapes = ((40, 128), (128,), (128, 384), (384,), (128, 384), (384,), (128, 10), (10,))
    for a in range(n_agents):
        o = 0
        for sh in shapes:
            n = int(np.prod(sh))
            if len(sh) == 2:
                lim = float(np.sqrt(6.0 / (sh[0] + sh[1])))
                out[a, o:o + n] = (torch.rand(n, generator=g) * 2 - 1) * lim
            o += n
    return out.to(device)


def gru_step(params: torch.Tensor, obs: torch.Tensor, h: torch.Tensor, n_actions: Sequence[int], seed: int, t: int,
             start: torch.Tensor = None, h_out: torch.Tensor = None, want_logits: bool = False,
             epoch: torch.Tensor = None, out: dict = None, obs_scale: torch.Tensor = None) -> dict:
    """One recurrent policy step: params [A, GRU_PARAMS], obs [A, n, 40], h [A, n, 128]
    (float32, device), start [n] uint8 or None -> actions, logp, value [A, n] and the new
    state in out["h"] (h_out, or h itself: updated in place)."""
    A, n = obs.shape[0], obs.shape[1]
    dev = obs.device
    if out is None:
        out = {"actions": torch.empty((A, n), dtype=torch.int32, device=dev),
               "logp": torch.empty((A, n), dtype=torch.float32, device=dev),
               "value": torch.empty((A, n), dtype=torch.float32, device=dev),
               "logits": torch.empty((A, n, 10), dtype=torch.float32, device=dev) if want_logits else None}
    ho = h if h_out is None else h_out
    na = (ctypes.c_int32 * A)(*[int(x) for x in n_actions])
    _check(_lib().lob_gru_step(_p(_f32(params)), _p(_f32(obs)), _p(_scale(obs_scale)), _p(_f32(h)), _p(_f32(ho)),
                               _p(None if start is None else start.to(torch.uint8).contiguous()), A, n, na, seed,
                               _p(epoch), t, _p(out.get("logits")), _p(out["actions"]), _p(out["logp"]),
                               _p(out["value"]), _stream()), "lob_gru_step")
    out["h"] = ho
    return out


def gru_workspace_bytes(T: int, m: int) -> int:
    return int(_lib().lob_gru_ppo_workspace_bytes(int(T), int(m)))


def gru_ppo_fwd_bwd(params, obs, start, h0, act, logp_old, adv, ret, v_old, n_actions, clip=0.2, c_v=0.5, c_e=0.01,
                    workspace=None, obs_scale=None):
    """Loss sums [4] and the gradient of the mean loss of m sequences of T steps:
    obs [T, m, 40], start [T, m] uint8, h0 [m, 128], act/logp_old/adv/ret/v_old [T, m]."""
    T, m = obs.shape[0], obs.shape[1]
    L = _lib()
    need = int(L.lob_gru_ppo_workspace_bytes(T, m))
    if workspace is None or workspace.numel() * 4 < need:
        workspace = torch.empty((need + 3) // 4, dtype=torch.float32, device=obs.device)
    loss = torch.empty(4, dtype=torch.float32, device=obs.device)
    grad = torch.empty(GRU_PARAMS, dtype=torch.float32, device=obs.device)
    _check(L.lob_gru_ppo_fwd_bwd(_p(_f32(params)), _p(_f32(obs)), _p(_scale(obs_scale)),
                                 _p(start.to(torch.uint8).contiguous()),
                                 _p(_f32(h0)), _p(act.to(torch.int32).contiguous()), _p(_f32(logp_old)),
                                 _p(_f32(adv)), _p(_f32(ret)), _p(_f32(v_old)), T, m, int(n_actions), clip, c_v, c_e,
                                 _p(workspace), workspace.numel() * 4, _p(loss), _p(grad), _stream()),
           "lob_gru_ppo_fwd_bwd")
    return loss, grad


class FusedGruPPOLoss(torch.autograd.Function):
    """Mean clipped-PPO loss of m whole sequences for the recurrent network; forward runs
    the fused recurrent kernels (forward through time keeping only the hidden states,
    backward through time recomputing the rest), which also produce the parameter
    gradient; backward scales it by the incoming gradient."""

    @staticmethod
    def forward(ctx, params, obs, start, h0, act, logp_old, adv, ret, v_old, n_actions, clip=0.2, c_v=0.5, c_e=0.01,
                obs_scale=None):
        loss, grad = gru_ppo_fwd_bwd(params.detach().contiguous(), obs, start, h0, act, logp_old, adv, ret, v_old,
                                     n_actions, clip, c_v, c_e, obs_scale=obs_scale)
        ctx.save_for_backward(grad)
        return loss[0] / (obs.shape[0] * obs.shape[1])

    @staticmethod
    def backward(ctx, g):
        (grad,) = ctx.saved_tensors
        return (g * grad,) + (None,) * 13


class FusedPPOLoss(torch.autograd.Function):
    """Mean clipped-PPO loss of one minibatch; forward runs the fused kernel, which also
    produces the parameter gradient (activations recomputed, none stored); backward
    scales that gradient by the incoming gradient."""

    @staticmethod
    def forward(ctx, params, obs, act, logp_old, adv, ret, v_old, n_actions, clip=0.2, c_v=0.5, c_e=0.01,
                obs_scale=None):
        loss, grad = ppo_fwd_bwd(params.detach().contiguous(), obs, act, logp_old, adv, ret, v_old, n_actions,
                                 clip, c_v, c_e, obs_scale=obs_scale)
        ctx.save_for_backward(grad)
        return loss[0] / obs.shape[0]

    @staticmethod
    def backward(ctx, g):
        (grad,) = ctx.saved_tensors
        return (g * grad,) + (None,) * 11
