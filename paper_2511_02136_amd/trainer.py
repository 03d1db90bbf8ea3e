"""IPPO on the batched LOB environment: learned-policy rollouts and PPO updates.

One independent actor-critic per agent (Sec. 4.2 of the paper: separate networks, no
shared weights): the feed-forward MLP, or the recurrent (GRU) network the paper trains
(Sec. 5.2.1), whose update runs over whole sequences (minibatches of envs) with the loss
taken back through time.  A rollout step is the policy forward (MFMA kernel, sampling
in-kernel) followed by one env step with the sampled actions; the whole T-step rollout
(reset included) can be captured once in a HIP graph and replayed, with a device counter
giving every replay fresh sampling noise.  The update runs GAE and, per agent, epochs of
shuffled minibatches through the fused clipped-PPO kernel (activations recomputed) and
torch's Adam.  Orchestration only: every step of the method runs in liblob's kernels.
"""
from __future__ import annotations

from typing import Optional

import torch

from . import ippo
from .lob import LobEnv, DeviceStream, N_ACTIONS

# Fixed input scaling of the 40 observation features (part of the policy, not the env):
# roughly the typical magnitude of each feature on the synthetic workloads.
OBS_SCALE = ([10.0, 10.0, 100.0] + [100.0] * 20 + [1e4, 1e4, 100.0, 100.0, 1e3, 1e3, 100.0, 10.0, 100.0, 1e7,
                                                    500.0, 128.0, 50.0, 50.0, 10.0, 50.0, 50.0])
assert len(OBS_SCALE) == 40


class IppoTrainer:
    def __init__(self, env: LobEnv, dstream: DeviceStream, book: dict, n_steps: int, seed: int = 0,
                 param_seed: int = 0, lr: float = 3e-4, epochs: int = 4, minibatches: int = 4, gamma: float = 0.99,
                 lam: float = 0.95, clip: float = 0.2, c_v: float = 0.5, c_e: float = 0.01, record_trades: bool = True,
                 network: str = "mlp", agent_streams: Optional[bool] = None):
        self.env, self.ds, self.book, self.T = env, dstream, book, n_steps
        self.A, self.N = env.n_agents, env.n_envs
        self.n_act = [N_ACTIONS[int(k)] for k in env.kinds]
        self.seed = seed
        self.epochs, self.minibatches = epochs, minibatches
        self.gamma, self.lam, self.clip, self.c_v, self.c_e = gamma, lam, clip, c_v, c_e
        dev = env.device
        if network not in ("mlp", "gru"):
            raise ValueError("network must be 'mlp' or 'gru'")
        self.network = network
        init = ippo.xavier_params if network == "mlp" else ippo.gru_init_params
        self.params = torch.nn.Parameter(init(self.A, param_seed, device=dev))
        self.opt = torch.optim.Adam([self.params], lr=lr)
        # the policy's input scaling, applied inside the policy and loss kernels
        self.inv_scale = (1.0 / torch.tensor(OBS_SCALE, dtype=torch.float32)).to(dev)
        T, A, N = n_steps, self.A, self.N
        # raw observations: [0] from the reset, [t + 1] written by the env step t itself
        self.obs = torch.empty((T + 1, A, N, 40), dtype=torch.float32, device=dev)
        self.pol = {"actions": torch.empty((T, A, N), dtype=torch.int32, device=dev),
                    "logp": torch.empty((T, A, N), dtype=torch.float32, device=dev),
                    "value": torch.empty((T, A, N), dtype=torch.float32, device=dev)}
        self.out = env._alloc_out(T, False, record_trades, None, dstream, actions_out=False)
        self.out["obs"] = self.obs[1:]
        self.cursor = torch.zeros(N, dtype=torch.int64, device=dev)
        self.epoch = torch.zeros(1, dtype=torch.int64, device=dev)
        # recurrent state of the GRU policy during the rollout (zero at the episode start)
        self.h = torch.zeros((A, N, ippo.GRU_HIDDEN), dtype=torch.float32, device=dev) if network == "gru" else None
        # each agent's loss calls on a stream of its own (False: all on the current one).
        # By default for the GRU only: its loss kernel fills 64 CUs per agent at 1024
        # sequences, so two agents side by side nearly halve the update (224 -> 135 ms on
        # the 4096-env workload); the MLP's fills the chip alone (31 ms one stream, 33 ms two).
        self.agent_streams = (network == "gru") if agent_streams is None else agent_streams
        self._streams = None
        self.graph: Optional[torch.cuda.CUDAGraph] = None

    # ---- rollout ----
    def _rollout_body(self):
        env, T = self.env, self.T
        ippo.counter_bump(self.epoch)
        env.reset(self.book)
        self.cursor.zero_()
        self.obs[0].copy_(env.observe())
        if self.h is not None:
            self.h.zero_()
        for t in range(T):
            pf = {k: v[t] for k, v in self.pol.items()}
            if self.h is None:
                ippo.policy_forward(self.params.detach(), self.obs[t], self.n_act, self.seed, t, epoch=self.epoch,
                                    out=pf, obs_scale=self.inv_scale)
            else:
                ippo.gru_step(self.params.detach(), self.obs[t], self.h, self.n_act, self.seed, t, epoch=self.epoch,
                              out=pf, obs_scale=self.inv_scale)
            view = {k: (v[t:t + 1] if k not in ("trades", "trade_off") and v is not None else v)
                    for k, v in self.out.items()}
            env.step(self.ds, pf["actions"], out=view, cursor=self.cursor)

    def rollout(self, use_graph: bool = False):
        """Reset and run T steps with the current policy; results stay in the buffers."""
        if not use_graph:
            self._rollout_body()
            return
        if self.graph is None:
            self.env.reset(self.book)
            self.env.plan(self.ds, self.T)
            # warm up on a side stream (library state, allocator), then capture
            s = torch.cuda.Stream()
            s.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(s):
                self._rollout_body()
            torch.cuda.current_stream().wait_stream(s)
            self.graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(self.graph):
                self._rollout_body()
        self.graph.replay()

    # ---- update ----
    def update(self) -> dict:
        T, A, N = self.T, self.A, self.N
        rew = self.out["reward"].reshape(T, A * N)
        val = self.pol["value"].reshape(T, A * N)
        done = self.out["done"].unsqueeze(1).expand(T, A, N).reshape(T, A * N).contiguous()
        adv, ret = ippo.gae(rew.contiguous(), val.contiguous(), done, torch.zeros(A * N, device=rew.device),
                            self.gamma, self.lam)
        adv, ret = adv.reshape(T, A, N), ret.reshape(T, A, N)
        if self.network == "gru":
            return self._update_gru(adv, ret)
        M = T * N
        mb = M // self.minibatches

        def agent_loss(a, idx):
            obs = self.obs[:T, a].reshape(M, 40)[idx].contiguous()
            act = self.pol["actions"][:, a].reshape(M)[idx].contiguous()
            lpo = self.pol["logp"][:, a].reshape(M)[idx].contiguous()
            ad = adv[:, a].reshape(M)[idx].contiguous()
            rt = ret[:, a].reshape(M)[idx].contiguous()
            vo = self.pol["value"][:, a].reshape(M)[idx].contiguous()
            return ippo.FusedPPOLoss.apply(self.params[a], obs, act, lpo, ad, rt, vo, self.n_act[a],
                                           self.clip, self.c_v, self.c_e, self.inv_scale)
        return self._epochs(M, mb, agent_loss)

    def _agent_streams(self):
        """One stream per agent (default priority): the agents' networks are independent,
        so their loss kernels of one minibatch may run side by side."""
        if self._streams is None:
            self._streams = [torch.cuda.Stream(device=self.env.device) for _ in range(self.A)]
        return self._streams

    def _epochs(self, n_items, mb, agent_loss) -> dict:
        """Epochs of shuffled minibatches; per minibatch every agent's fused loss call is
        issued on its own stream (forward and, by autograd's stream rule, backward), the
        losses summed on the current stream, then one Adam step over all networks."""
        dev = self.params.device
        streams = self._agent_streams() if self.agent_streams else None
        stats = {"loss": 0.0, "minibatches": 0}
        for _ in range(self.epochs):
            perms = [torch.randperm(n_items, device=dev) for _ in range(self.A)]
            for k in range(self.minibatches):
                self.opt.zero_grad(set_to_none=True)
                main = torch.cuda.current_stream(dev)
                losses = []
                for a in range(self.A):
                    idx = perms[a][k * mb:(k + 1) * mb]
                    if streams is None:
                        losses.append(agent_loss(a, idx))
                        continue
                    streams[a].wait_stream(main)
                    with torch.cuda.stream(streams[a]):
                        losses.append(agent_loss(a, idx))
                for st in streams or ():
                    main.wait_stream(st)
                total = losses[0]
                for l in losses[1:]:
                    total = total + l
                total.backward()
                self.opt.step()
                stats["loss"] += float(total.detach())
                stats["minibatches"] += 1
                del losses, total  # the graph of this minibatch, before the next one's forward
        stats["loss"] /= max(1, stats["minibatches"])
        return stats

    def _update_gru(self, adv, ret) -> dict:
        """Epochs of minibatches of whole sequences (envs), the loss back through time."""
        T, N = self.T, self.N
        dev = adv.device
        mb = N // self.minibatches
        start = torch.zeros((T, mb), dtype=torch.uint8, device=dev)
        start[0] = 1  # the rollout is one episode from its reset
        h0 = torch.zeros((mb, ippo.GRU_HIDDEN), dtype=torch.float32, device=dev)

        def agent_loss(a, idx):
            obs = self.obs[:T, a][:, idx].contiguous()
            act = self.pol["actions"][:, a][:, idx].contiguous()
            lpo = self.pol["logp"][:, a][:, idx].contiguous()
            ad = adv[:, a][:, idx].contiguous()
            rt = ret[:, a][:, idx].contiguous()
            vo = self.pol["value"][:, a][:, idx].contiguous()
            return ippo.FusedGruPPOLoss.apply(self.params[a], obs, start, h0, act, lpo, ad, rt, vo,
                                              self.n_act[a], self.clip, self.c_v, self.c_e, self.inv_scale)
        return self._epochs(N, mb, agent_loss)
