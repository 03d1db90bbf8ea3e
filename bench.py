"""Benchmark: batched LOB environment rollout on one MI355X.

Workload: 8192 envs with uneven shapes (per-side book capacity uniform in
{50,100,200,400}, messages per step uniform in 1..400 per env), execution + market-making
agent under the in-kernel random policy, 128-step episodes; synthetic MBO streams.
One benchmark step = reset + one 128-step rollout of every env (persistent form: books
LDS-resident for all steps, the schedule picked by the autotuner before timing, the
rollout captured once in a HIP graph and replayed), all outputs written (trades, fills,
rewards, observations).

Prints one JSON line.  value = replayed MBO messages per second (whole job); the line
also carries env-steps/s, the plain per-step form's throughput for comparison, the
roofline of the env kernel and the CPU oracle's throughput on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOAD = "uneven8192"


def algorithmic_bytes(n_msgs, n_trades, n_envs, n_agents, n_steps, book_slots):
    """Bytes the method must move for one rollout: messages in (7 x int32), trade
    records out (8 x int32), per env-step outputs (obs 40 fp32, reward fp32, fills
    4 x int64 and action int32 per agent; done u8, trade count int32), and each book's
    live orders in once and out once (6 x int32 each way)."""
    per_env_step = n_agents * (160 + 4 + 32 + 4) + 1 + 4
    return 28 * n_msgs + 32 * n_trades + per_env_step * n_envs * n_steps + 48 * book_slots


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for f in ("paper_2511_02136_amd/csrc/lob_env.hip", "paper_2511_02136_amd/csrc/lob_device.h"):
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str):
    """HBM bytes per rollout from the committed rocprofv3 counter summary, or None when
    the summary is missing or was taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", f"k_env_{workload}_hbm_bytes.md")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        for line in fh:
            if line.startswith("traffic_json: "):
                t = json.loads(line[len("traffic_json: "):])
                if t.get("source_sha") == kernel_source_sha():
                    return float(t["traffic_bytes"])
    return None


# one SALU instruction per CU per cycle (each SIMD issues one every 4 cycles)
N_CU, CLOCK_HZ = 256, 2.4e9


def measured_issue(workload: str, n_msgs: int, kernel_ms: float):
    """Issue view of k_env from the committed instruction-mix summary (rocprofv3
    SQ_INSTS_* counters), or None when it is missing or from a different kernel source:
    the time the SALU instructions alone need at one per CU per cycle, and the LDS
    instructions at one per CU per cycle, as fractions of the measured kernel time."""
    path = os.path.join(ROOT, "profiles", f"k_env_{workload}_instruction_mix.md")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        for line in fh:
            if line.startswith("mix_json: "):
                m = json.loads(line[len("mix_json: "):])
                if m.get("source_sha") != kernel_source_sha():
                    return None
                salu_ms = m["salu_per_msg"] * n_msgs / (N_CU * CLOCK_HZ) * 1e3
                lds_ms = m["lds_per_msg"] * n_msgs / (N_CU * CLOCK_HZ) * 1e3
                return {"salu_per_msg": m["salu_per_msg"], "valu_per_msg": m["valu_per_msg"],
                        "lds_per_msg": m["lds_per_msg"], "salu_issue_ms": salu_ms,
                        "salu_issue_frac": salu_ms / kernel_ms, "lds_issue_ms": lds_ms,
                        "lds_issue_frac": lds_ms / kernel_ms}
    return None


def copy_bandwidth(nbytes: int = 1 << 30, reps: int = 5) -> float:
    """Device-to-device copy bandwidth on this GPU (read + write bytes per second, GB/s)."""
    import torch
    src = torch.empty(nbytes // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    del src, dst
    return 2 * nbytes * reps / (ms / 1e3) / 1e9


def workload_figures(name: str, reps: int = 2) -> dict:
    """Persistent-rollout throughput of another workload (all outputs written), plus the
    oracle on one host thread over a bounded sample of its envs."""
    import torch
    from paper_2511_02136_amd import synth
    from paper_2511_02136_amd.lob import LobEnv, DeviceStream
    w = synth.WORKLOADS[name]
    s = synth.generate(w)
    cpu1 = cpu_baseline(w, s, budget_s=6.0, threads=1)
    ds = DeviceStream.from_host(s)
    n_msgs = s.n_msgs
    book = {k: torch.from_numpy(v).cuda() for k, v in s.book.items()}
    caps = s.caps
    del s
    env = LobEnv(caps, w.max_cap, w.agents, w.ep_len, w.seed)
    toff = ds.trade_regions(env.caps, 0, w.n_steps, len(w.agents))
    out = env._alloc_out(w.n_steps, True, True, toff, ds)
    env.reset(book)
    env.plan(ds, w.n_steps)
    env.reset(book)
    env.rollout(ds, w.n_steps, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        env.reset(book)
        env.rollout(ds, w.n_steps, out=out)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    all_msgs = int(env.state()["counters"][:, 0].sum().item())
    return {"workload": name, "n_envs": w.n_envs, "n_steps": w.n_steps, "replay_msgs": n_msgs,
            "ms_per_rollout": ms, "msgs_per_s": n_msgs / (ms / 1e3),
            "all_msgs_per_s": all_msgs / (ms / 1e3),
            "env_steps_per_s": w.n_envs * w.n_steps / (ms / 1e3), "cpu_oracle_1thread": cpu1}


def cpu_baseline(w, stream, budget_s=15.0, threads=None):
    """The CPU oracle on a bounded sample of the same workload (first envs, all steps)."""
    import oracle
    from paper_2511_02136_amd import synth
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from helpers import subset_stream
    if threads is None:
        threads = max(1, min(16, os.cpu_count() or 1))
    n = min(w.n_envs, 64 if threads > 1 else 4)
    while True:
        envs = np.arange(n)
        hs, book, caps = subset_stream(stream, envs)
        o = oracle.OracleEnvs(caps, w.max_cap, synth.agent_kinds(w.agents), w.ep_len, w.seed, env_ids=envs)
        o.reset(book)
        t0 = time.perf_counter()
        o.step(hs, n_steps=w.n_steps, threads=threads, record_trades=True)
        dt = time.perf_counter() - t0
        msgs = int(hs.off[:, w.n_steps].sum() - hs.off[:, 0].sum())
        if dt >= budget_s / 4 or n >= w.n_envs:
            return {"value": msgs / dt, "unit": "msgs/s", "cores": threads, "kind": "oracle",
                    "env_steps_per_s": n * w.n_steps / dt,
                    "sample": f"{n} of {w.n_envs} envs x {w.n_steps} steps ({msgs} msgs), {dt:.2f} s"}
        n = min(w.n_envs, n * max(2, int(budget_s / 4 / max(dt, 1e-3))))

# fused clipped-PPO forward+backward per sample: forward 40x256 + 256x256 + 256x10 MACs,
# backward the weight gradients of all three layers and the input gradients of layers 2
# and 3 (none for the observation); 2 FLOP per MAC
PPO_FLOP_PER_SAMPLE = 2 * ((40 * 256 + 256 * 256 + 256 * 10) * 2 + 256 * 256 + 256 * 10)
FP32_MFMA_PEAK_TFLOPS = 157.3
# recurrent network per sample: forward 40x128 + 128x384 + 128x384 + 128x10 MACs (embedding,
# input and recurrent gate products, head); backward the input gradients of the head, the
# recurrent and the gate products (none for the observation) and every weight gradient;
# 2 FLOP per MAC.  The forward pass the kernel runs a second time (recomputation) is not
# counted.
GRU_FWD_MACS = 40 * 128 + 2 * 128 * 384 + 128 * 10
GRU_FLOP_PER_SAMPLE = 2 * (GRU_FWD_MACS + (128 * 10 + 2 * 128 * 384) + GRU_FWD_MACS)


def gru_bench(reps: int = 3):
    """ippo4096 with the recurrent (GRU) actor-critic: graph-captured learned-policy rollout,
    one update over whole sequences (4 epochs x 4 minibatches of 1024 envs x 128 steps per
    agent) and one fused GRU loss call on a full minibatch, with its MFMA roofline."""
    import torch
    from paper_2511_02136_amd import synth, ippo
    from paper_2511_02136_amd.lob import LobEnv, DeviceStream
    from paper_2511_02136_amd.trainer import IppoTrainer
    w = synth.WORKLOADS["ippo4096"]
    s = synth.generate(w)
    ds = DeviceStream.from_host(s)
    env = LobEnv(s.caps, w.max_cap, w.agents, w.ep_len, w.seed)
    book = {k: torch.from_numpy(v).cuda() for k, v in s.book.items()}
    tr = IppoTrainer(env, ds, book, w.n_steps, seed=w.seed, network="gru")
    tr.rollout(use_graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        tr.rollout(use_graph=True)
    torch.cuda.synchronize()
    roll_ms = (time.perf_counter() - t0) * 1e3 / reps
    tr.update()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tr.update()
    torch.cuda.synchronize()
    upd_ms = (time.perf_counter() - t0) * 1e3
    T, N = w.n_steps, w.n_envs
    m = N // tr.minibatches
    obs = tr.obs[:T, 0][:, :m].contiguous()
    start = torch.zeros((T, m), dtype=torch.uint8, device="cuda")
    start[0] = 1
    h0 = torch.zeros((m, ippo.GRU_HIDDEN), dtype=torch.float32, device="cuda")
    act = tr.pol["actions"][:, 0][:, :m].contiguous()
    lpo = tr.pol["logp"][:, 0][:, :m].contiguous()
    val = tr.pol["value"][:, 0][:, :m].contiguous()
    adv = torch.randn((T, m), device="cuda")
    ret = val + 0.1 * torch.randn((T, m), device="cuda")
    prm = tr.params.detach()[0].contiguous()
    ws = torch.empty((ippo.gru_workspace_bytes(T, m) + 3) // 4, dtype=torch.float32, device="cuda")
    args = (prm, obs, start, h0, act, lpo, adv, ret, val, tr.n_act[0])
    ippo.gru_ppo_fwd_bwd(*args, workspace=ws, obs_scale=tr.inv_scale)
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    n_calls = 5
    e0.record(st)
    for _ in range(n_calls):
        ippo.gru_ppo_fwd_bwd(*args, workspace=ws, obs_scale=tr.inv_scale)
    e1.record(st)
    torch.cuda.synchronize()
    call_ms = e0.elapsed_time(e1) / n_calls
    tflops = T * m * GRU_FLOP_PER_SAMPLE / (call_ms / 1e3) / 1e12
    return {"workload": f"ippo4096: {N} envs x {T} steps, 2 agents, GRU 40-128-GRU(128)-(9+1) fp32",
            "rollout_ms": roll_ms, "rollout_env_steps_per_s": N * T / (roll_ms / 1e3), "update_ms": upd_ms,
            "update": "GAE + 4 epochs x 4 minibatches (1024 sequences of 128 steps) x 2 agents + Adam",
            "gru_ppo_fwd_bwd_call": {"sequences": m, "steps": T, "samples": T * m, "ms": call_ms,
                                     "flop_per_sample": GRU_FLOP_PER_SAMPLE,
                                     "launches": "k_gru_prep, k_gru_in, k_gru_fwd, k_gru_head, k_gru_bwd, "
                                                 "k_gru_de, k_gru_dw, k_reduce_chunks, k_reduce_out, k_gru_loss",
                                     "roofline": {"bound": "mfma", "achieved": tflops, "peak": FP32_MFMA_PEAK_TFLOPS,
                                                  "unit": "TFLOP/s", "frac": tflops / FP32_MFMA_PEAK_TFLOPS}}}


def ippo_bench(reps: int = 3):
    """ippo4096: 4096 envs x 128 steps, two actor-critics.  Times the graph-captured
    learned-policy rollout, one PPO update (4 epochs x 4 minibatches per agent) and one
    fused PPO forward+backward call (fused kernel and its two reduction launches) on one
    full minibatch (131072 samples)."""
    import torch
    from paper_2511_02136_amd import synth, ippo
    from paper_2511_02136_amd.lob import LobEnv, DeviceStream
    from paper_2511_02136_amd.trainer import IppoTrainer
    w = synth.WORKLOADS["ippo4096"]
    s = synth.generate(w)
    ds = DeviceStream.from_host(s)
    env = LobEnv(s.caps, w.max_cap, w.agents, w.ep_len, w.seed)
    book = {k: torch.from_numpy(v).cuda() for k, v in s.book.items()}
    tr = IppoTrainer(env, ds, book, w.n_steps, seed=w.seed)
    tr.rollout(use_graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        tr.rollout(use_graph=True)
    torch.cuda.synchronize()
    roll_ms = (time.perf_counter() - t0) * 1e3 / reps
    tr.update()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tr.update()
    torch.cuda.synchronize()
    upd_ms = (time.perf_counter() - t0) * 1e3
    # the fused kernel on one minibatch of agent 0's rollout data
    T, N = w.n_steps, w.n_envs
    m = T * N // tr.minibatches
    obs = tr.obs[:T, 0].reshape(T * N, 40)[:m].contiguous()
    act = tr.pol["actions"][:, 0].reshape(-1)[:m].contiguous()
    lpo = tr.pol["logp"][:, 0].reshape(-1)[:m].contiguous()
    val = tr.pol["value"][:, 0].reshape(-1)[:m].contiguous()
    adv = torch.randn(m, device="cuda")
    ret = val + 0.1 * torch.randn(m, device="cuda")
    prm = tr.params.detach()[0].contiguous()
    ws = torch.empty((ippo.workspace_bytes(m) + 3) // 4, dtype=torch.float32, device="cuda")
    ippo.ppo_fwd_bwd(prm, obs, act, lpo, adv, ret, val, tr.n_act[0], workspace=ws, obs_scale=tr.inv_scale)
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    n_calls = 10
    e0.record(st)
    for _ in range(n_calls):
        ippo.ppo_fwd_bwd(prm, obs, act, lpo, adv, ret, val, tr.n_act[0], workspace=ws, obs_scale=tr.inv_scale)
    e1.record(st)
    torch.cuda.synchronize()
    ppo_ms = e0.elapsed_time(e1) / n_calls
    tflops = m * PPO_FLOP_PER_SAMPLE / (ppo_ms / 1e3) / 1e12
    env_steps = N * T
    return {"workload": f"ippo4096: {N} envs x {T} steps, 2 agents (exec, mm), MLP 40-256-256-(9+1) fp32",
            "rollout_ms": roll_ms, "rollout_env_steps_per_s": env_steps / (roll_ms / 1e3),
            "update_ms": upd_ms, "update": "GAE + 4 epochs x 4 minibatches x 2 agents of fused PPO + Adam",
            "ppo_fwd_bwd_call": {"samples": m, "ms": ppo_ms, "flop_per_sample": PPO_FLOP_PER_SAMPLE,
                                 "launches": "k_w2t, k_ppo_fwd_bwd, k_reduce_chunks, k_reduce_final",
                           "roofline": {"bound": "mfma", "achieved": tflops, "peak": FP32_MFMA_PEAK_TFLOPS,
                                        "unit": "TFLOP/s", "frac": tflops / FP32_MFMA_PEAK_TFLOPS}}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=WORKLOAD)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain per-step form")
    ap.add_argument("--no-ippo", action="store_true", help="skip the IPPO rollout/update figures")
    ap.add_argument("--configs", default="replay1",
                    help="comma-separated extra workloads to report (default replay1; also uniform4096, large16384)")
    ap.add_argument("--ippo-only", action="store_true",
                    help="only the IPPO figures (profiling aid; prints them as one JSON object)")
    ap.add_argument("--gru-only", action="store_true",
                    help="only the recurrent actor-critic figures (profiling aid; one JSON object)")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the schedule autotuner (the default plan and balance share instead)")
    ap.add_argument("--eager", action="store_true",
                    help="time eager rollouts instead of replays of the captured HIP graph")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first copy 256 MiB device-to-device, by the blit copy and by an elementwise kernel "
                         "(calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the env step shards by env "
              "with no exchange, and this benchmark measures one GPU's share.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2511_02136_amd import synth
    from paper_2511_02136_amd.lob import LobEnv, DeviceStream

    if args.copy_probe:
        # HBM byte-counter calibration: 256 MiB read and 256 MiB written, once by the
        # runtime's blit copy and once by an ordinary elementwise kernel (x * 1)
        src = torch.ones(64 << 20, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        torch.mul(src, 1, out=dst)
        torch.cuda.synchronize()
        del src, dst
    if args.ippo_only:
        print(json.dumps({"ippo": ippo_bench()}), flush=True)
        return
    if args.gru_only:
        print(json.dumps({"ippo_gru": gru_bench()}), flush=True)
        return
    w = synth.WORKLOADS[args.workload]
    print(f"[bench] generating {w.name}", file=sys.stderr, flush=True)
    s = synth.generate(w)
    ds = DeviceStream.from_host(s)
    env = LobEnv(s.caps, w.max_cap, w.agents, w.ep_len, w.seed)
    book = {k: torch.from_numpy(v).cuda() for k, v in s.book.items()}
    toff = ds.trade_regions(env.caps, 0, w.n_steps, len(w.agents))
    out = env._alloc_out(w.n_steps, True, True, toff, ds)
    stream = torch.cuda.current_stream()
    env.reset(book)
    if not args.no_tune:
        # the tuner times schedules on this rollout (state restored), outside the timed region
        print("[bench] autotune", file=sys.stderr, flush=True)
        env.autotune(ds, w.n_steps, out=out)
    else:
        env.plan(ds, w.n_steps)
    schedule = env.schedule()
    torch.cuda.synchronize()
    graph = None
    if not args.eager:
        # the rollout (every class launch, the staggered starts, the queue counters cleared by a
        # kernel) captured once in a HIP graph; the reset before each replay stays eager
        env.reset(book)
        env.rollout(ds, w.n_steps, out=out)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        env.reset(book)
        torch.cuda.synchronize()
        with torch.cuda.graph(graph):
            env.rollout(ds, w.n_steps, out=out)
        torch.cuda.synchronize()

    def one_rollout(ev=None):
        env.reset(book)
        if ev is not None:
            ev.record(stream)
        if graph is not None:
            graph.replay()
        else:
            env.rollout(ds, w.n_steps, out=out)

    print(f"[bench] warmup {args.warmup}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        one_rollout()
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    mids = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    print(f"[bench] timing {args.steps} rollouts", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        starts[k].record(stream)
        one_rollout(mids[k])
        ends[k].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = wall * 1e3 / args.steps
    kernel_ms = float(np.mean([mids[k].elapsed_time(ends[k]) for k in range(args.steps)]))

    median_ms = float(np.median([starts[k].elapsed_time(ends[k]) for k in range(args.steps)]))
    n_msgs = s.n_msgs
    all_msgs = int(env.state()["counters"][:, 0].sum().item())  # every processed message, agents' too
    n_trades = int(out["n_trades"].sum().item())
    book_slots = int(s.book["n"].sum()) + int(env.books()["n"].sum().item())
    book_slots //= 2
    env_steps = w.n_envs * w.n_steps
    msgs_per_s = n_msgs / (ms_step / 1e3)
    steps_per_s = env_steps / (ms_step / 1e3)
    alg = algorithmic_bytes(n_msgs, n_trades, w.n_envs, len(w.agents), w.n_steps, book_slots)
    achieved = alg / (kernel_ms / 1e3) / 1e9

    # sampled parity of the timed rollout against the oracle (outside the timed region)
    parity = "skipped"
    try:
        import oracle  # noqa: F401
        sys.path.insert(0, os.path.join(ROOT, "tests"))
        from helpers import subset_stream
        from gpu_compare import assert_same_outputs
        sample = np.array([0, 1, w.n_envs // 2, w.n_envs - 1])
        hs, bk, caps = subset_stream(s, sample)
        o = oracle.OracleEnvs(caps, w.max_cap, synth.agent_kinds(w.agents), w.ep_len, w.seed, env_ids=sample)
        o.reset(bk)
        acts = np.ascontiguousarray(out["actions"].cpu().numpy()[:, :, sample])
        ref = o.step(hs, n_steps=w.n_steps, actions=acts)
        g = {k: v for k, v in out.items() if k not in ("trades",)}
        r = dict(ref)
        r["trades"] = None
        assert_same_outputs(g, r, w.n_steps, envs=sample, what="bench")
        goff = toff.cpu().numpy()
        for j, e in enumerate(sample):
            cnt = int(ref["n_trades"][:, j].sum())
            a = out["trades"][goff[e]: goff[e] + cnt].cpu().numpy()
            b = ref["trades"][ref["trade_off"][j]: ref["trade_off"][j] + cnt]
            assert np.array_equal(a, b)
        parity = "bit-exact on 4 sampled envs"
    except AssertionError as ex:
        parity = f"MISMATCH: {ex}"

    # context only, not the value: the same rollouts each started on an idle GPU (host
    # synchronised before each).  Rollouts queued back to back, as timed above, run in
    # one of two modes from one rollout to the next; from an idle GPU they do not.
    # (a context leg like the per-step forms: skipped with --no-plain, as in profiling runs)
    from_idle = []
    if not args.no_plain:
        print("[bench] rollouts started from an idle GPU (context)", file=sys.stderr, flush=True)
        for _ in range(args.steps):
            env.reset(book)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            env.rollout(ds, w.n_steps, out=out)
            e1.record(stream)
            torch.cuda.synchronize()
            from_idle.append(e0.elapsed_time(e1))

    copy_gbs = copy_bandwidth()
    traffic = measured_traffic(w.name)

    plain = plain_padded = None
    if not args.no_plain:
        # plain per-step form: one launch per step, books through HBM every step
        print("[bench] plain per-step form", file=sys.stderr, flush=True)
        cursor = torch.zeros(w.n_envs, dtype=torch.int64, device="cuda")

        def plain_rollout():
            env.reset(book)
            cursor.zero_()
            for t in range(w.n_steps):
                view = {k: (v[t:t + 1] if k not in ("trades", "trade_off") and v is not None else v)
                        for k, v in out.items()}
                env.step(ds, None, out=view, cursor=cursor)

        plain_rollout()
        torch.cuda.synchronize()
        reps = max(1, min(args.steps, 3))
        t1 = time.perf_counter()
        for _ in range(reps):
            plain_rollout()
        torch.cuda.synchronize()
        pms = (time.perf_counter() - t1) * 1e3 / reps
        plain = {"ms_per_rollout": pms, "env_steps_per_s": env_steps / (pms / 1e3),
                 "msgs_per_s": n_msgs / (pms / 1e3), "persistent_speedup": pms / ms_step}

        # batching ablation: the same per-step launches with every env in one class padded
        # to the largest capacity, dispatched in env order (no capacity classes, no plan)
        print("[bench] padded per-step form", file=sys.stderr, flush=True)
        env.set_padded(True)
        plain_rollout()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(reps):
            plain_rollout()
        torch.cuda.synchronize()
        qms = (time.perf_counter() - t1) * 1e3 / reps
        env.set_padded(False)
        plain_padded = {"ms_per_rollout": qms, "env_steps_per_s": env_steps / (qms / 1e3),
                        "msgs_per_s": n_msgs / (qms / 1e3), "persistent_speedup": qms / ms_step}

    ippo_res = None
    if not args.no_ippo:
        print("[bench] ippo4096: learned-policy rollout, PPO update", file=sys.stderr, flush=True)
        del out, env, ds
        torch.cuda.empty_cache()
        ippo_res = ippo_bench()
        torch.cuda.empty_cache()
        print("[bench] ippo4096 with the recurrent network", file=sys.stderr, flush=True)
        ippo_res["gru"] = gru_bench()

    cpu = None
    if not args.no_cpu:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(w, s)
        one = cpu_baseline(w, s, budget_s=8.0, threads=1)
        cpu["one_thread"] = {"value": one["value"], "sample": one["sample"]}
        cpu["host_cpus"] = os.cpu_count()

    extra = None
    if args.configs:
        extra = []
        for name in [c for c in args.configs.split(",") if c]:
            print(f"[bench] workload {name}", file=sys.stderr, flush=True)
            torch.cuda.empty_cache()
            extra.append(workload_figures(name))

    line = {
        "metric": "MBO messages/sec and env-steps/sec at 8192 envs, bit-exact vs oracle",
        "value": msgs_per_s,
        "unit": "msgs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.n_envs} envs, cap U{{50,100,200,400}}, msgs/step U{{1..400}}, "
                               f"{w.n_steps} steps, agents exec+mm, random policy",
                   "n_envs": w.n_envs, "n_steps": w.n_steps, "n_msgs": n_msgs,
                   "form": "eager rollout" if graph is None else "replay of the captured HIP graph",
                   "schedule": "default plan" if args.no_tune else "autotuned before timing"},
        "env_steps_per_s": steps_per_s,
        "all_msgs_per_s": all_msgs / (ms_step / 1e3),
        "median_ms_per_step": median_ms,
        "rollout_ms_timed": [round(mids[k].elapsed_time(ends[k]), 2) for k in range(args.steps)],
        "rollout_ms_from_idle": [round(t, 2) for t in from_idle],
        "trades": n_trades,
        "parity": parity,
        "schedule": schedule,
        "plain_form": plain,
        "plain_padded": plain_padded,
        "ippo": ippo_res,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_gbs": None if traffic is None else traffic / (kernel_ms / 1e3) / 1e9,
                     "copy_gbs": copy_gbs, "frac_vs_copy": achieved / copy_gbs,
                     "kernel": "k_env (persistent rollout, all capacity classes)",
                     "kernel_ms": kernel_ms, "algorithmic_bytes": alg,
                     "scalar_issue": measured_issue(w.name, n_msgs, kernel_ms)},
        "cpu_baseline": cpu,
        "other_workloads": extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
