/*
 * liblob — batched limit-order-book environment step for MI355X (gfx950).
 *
 * The hot path of the JaxMARL-HFT environment (arXiv 2511.02136, Sec. 4): for thousands
 * of parallel environments, one env-step
 *   1. converts each agent's discrete action into order-book messages, cancelling the
 *      agent's earlier unmatched orders unless it quotes again at the same price level
 *      (Sec. 4, step 1; agent types of Sec. 4.1),
 *   2. shuffles the agents' new orders (Sec. 4, step 2),
 *   3. concatenates [cancels, shuffled orders, replayed market-by-order messages]
 *      (Sec. 4, step 3),
 *   4. processes them in sequence against a fixed-capacity price-time-priority book,
 *      recording trades (Sec. 4, step 4; Sec. 2.1; capacity from Table 2),
 *   5. computes fills, rewards (Eq. 2-4), done flags and observations (Sec. 4, step 5).
 *
 * Conventions
 *   - Every pointer named *_d / documented "device" is device memory owned by the caller
 *     (e.g. a torch tensor's data_ptr()); host pointers are read during the call only.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Calls that
 *     launch work are asynchronous on that stream; arguments are validated on the host
 *     first and a negative code is returned synchronously on error (nothing launched).
 *   - Device-side conditions (cancel misses, evictions, drops, unfilled market orders,
 *     trade records that did not fit) are counted per env, never turned into errors.
 *   - Integer work (books, trades, fills, counters) is exact.  Rewards are one double
 *     expression per agent rounded once to float; observations are integers converted
 *     to float with round-to-nearest-even.
 *
 * Message encoding (structure of arrays, int32 each, one entry per message):
 *   ts    = type | (side << 8); type 1 LIMIT, 2 PARTIAL_CANCEL, 3 DELETE, 4 MARKET
 *           (immediate-or-cancel, no price limit), 5 EXECUTE (a replayed execution of
 *           the resting order named by oid on `side`: min(qty, its qty) trades at its
 *           price against an anonymous aggressor of the other side, oid 0 and tid 0, and
 *           the rest keeps its priority; a missing id counts as a miss), 6 IGNORED (a
 *           replayed message the book does not act on: hidden executions, cross trades,
 *           trading halts; counted); side 0 buy, 1 sell; other types are counted as bad
 *           and ignored.
 *   price (ticks), qty (> 0), oid (order id; cancels name the order by id on their
 *   side), tid (trader id; agents are tid 1..n_agents, replay data must not use them),
 *   tsec, tns (time payload, not used for priority: arrival order is time priority).
 * Replay message ids must stay below 2^30 (agent order ids have bit 30 set).
 */
#ifndef LOB_H
#define LOB_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    LOB_OK = 0,
    LOB_EINVAL = -1,       /* a bad argument (sizes, NULL pointers, ranges) */
    LOB_ENOMEM = -2,       /* device allocation failed */
    LOB_EHIP = -3,         /* a HIP runtime call failed */
    LOB_ESTATE = -4,       /* call order: no reset yet, or the episode/stream is exhausted */
    LOB_EUNSUPPORTED = -5  /* a configuration the library does not support */
};

#define LOB_LIMIT 1
#define LOB_PARTIAL_CANCEL 2
#define LOB_DELETE 3
#define LOB_MARKET 4
#define LOB_OBS_DIM 40
#define LOB_TRADE_WORDS 8
#define LOB_N_COUNTERS 11
#define LOB_ENV_STATE_WORDS 12
#define LOB_AGENT_STATE_WORDS 6
#define LOB_MAX_AGENTS 4
#define LOB_MAX_CAP 1024

/* agent kinds (Sec. 4.1) */
#define LOB_AGENT_EXEC 0 /* order execution, sell task; 9 actions */
#define LOB_AGENT_MM 1   /* market making, fixed-quantity action space; 9 actions */
#define LOB_AGENT_DIR 2  /* directional trading; 3 actions */
#define LOB_AGENT_MM_BUYSELL 3 /* market making as LOB_AGENT_MM, rewarded by the buy-sell
                                * PnL (Eq. 4) minus the quadratic inventory penalty */
/* The market maker's other action spaces of Sec. 4.1.1 (rewarded as LOB_AGENT_MM, Eq. 3
 * with the quadratic penalty).  The paper gives no tables; readings: */
#define LOB_AGENT_MM_SPREADSKEW 4 /* spread-skew table, 9 actions, always two-sided: spread
                                   * S = 1, 3, 5 ticks around the mid times skew k = -1, 0, +1
                                   * (action 3 * (index of S) + index of k): bid =
                                   * floor((bb + ba - S) / 2) + k, ask = ceil((bb + ba + S) / 2)
                                   * + k, never crossing the step-start touch */
#define LOB_AGENT_MM_AVST 5       /* Avellaneda-Stoikov quotes with the risk aversion as the
                                   * action, 9 actions: gamma = avst_gamma * 2^(a - 4);
                                   * reservation price mid - q gamma sigma^2 (T - t), spread
                                   * gamma sigma^2 (T - t) + (2 / gamma) ln(1 + gamma / kappa),
                                   * q = inventory / mm_q, T - t the steps left including the
                                   * current one; bid = floor(r - spread / 2), ask = ceil(r +
                                   * spread / 2), one quote of mm_q per side, never crossing the
                                   * step-start touch; evaluated in double */
/* The baselines the learned agents are evaluated against (Sec. 5.2.2); their action is
 * not used (one action): */
#define LOB_AGENT_EXEC_TWAP 6     /* execution by TWAP: each step sells the shortfall to
                                   * ceil(exec_task (t + 1) / episode_len) executed (at most the
                                   * remainder) with one limit order at the step-start best bid;
                                   * rewarded as LOB_AGENT_EXEC (Eq. 2 and the end penalty) */
#define LOB_AGENT_MM_AS 7         /* the Avellaneda-Stoikov market maker: LOB_AGENT_MM_AVST
                                   * always at gamma = avst_gamma (action 4) */

typedef struct lob_ctx lob_ctx;

/* Environment configuration (host struct, copied by lob_init). */
typedef struct {
    int32_t n_envs;            /* >= 1 */
    int32_t n_agents;          /* 0..LOB_MAX_AGENTS; agent i has tid i+1 */
    int32_t max_cap;           /* 1..LOB_MAX_CAP: stride of book arrays, >= every cap */
    int32_t episode_len;       /* steps per episode (done on the last) */
    const int32_t *cap;        /* host [n_envs]: per-side capacity of each env's book */
    const int32_t *agent_kind; /* host [n_agents]: LOB_AGENT_* */
    uint64_t seed;             /* shuffle keys and random-policy actions */
    int32_t exec_task;         /* shares the execution agent sells per episode */
    int32_t exec_q0;           /* execution order quantity */
    int32_t mm_q;              /* market-maker quote quantity */
    int32_t dir_q;             /* directional order quantity */
    float exec_penalty;        /* end-of-episode penalty per unfilled share, times P_init */
    float mm_lambda;           /* Spooner weight of positive inventory PnL (Eq. 3) */
    float mm_rho;              /* quadratic inventory penalty factor */
    uint32_t flags;            /* reserved, must be 0 */
    /* Avellaneda-Stoikov quotes (LOB_AGENT_MM_AVST, LOB_AGENT_MM_AS; ignored otherwise):
     * base risk aversion gamma0 > 0, price variance per step sigma^2 >= 0 (ticks^2),
     * order-arrival decay kappa > 0 (per tick); mm_q must then be > 0 (LOB_EINVAL) */
    float avst_gamma, avst_sigma2, avst_kappa;
} lob_config;

/* A market-by-order stream in CSR form (device arrays).  Env e's messages of step t are
 * entries off[e*(n_steps+1)+t] .. off[e*(n_steps+1)+t+1]-1 of the seven arrays. */
typedef struct {
    const int32_t *ts, *price, *qty, *oid, *tid, *tsec, *tns; /* device [n_msgs] */
    const int64_t *off;                                       /* device [n_envs][n_steps+1] */
    int32_t n_steps;                                          /* CSR rows per env */
    int64_t n_msgs;                                           /* entries of each array */
} lob_msgs;

/* Books in canonical layout (device arrays): field[e][side][slot] with side 0 = bids,
 * 1 = asks, slots 0..n-1 in priority order (best price first, then arrival), unused slots
 * zero on export; n[e][side] order counts. */
typedef struct {
    int32_t *price, *qty, *oid, *tid, *tsec, *tns; /* device [n_envs][2][max_cap] */
    int32_t *n;                                    /* device [n_envs][2] */
} lob_books;

/* Outputs of lob_step / lob_rollout for n_steps steps (device arrays).
 * trade record (8 int32): price, qty, aggressor oid, resting oid, aggressor tid,
 *   resting tid, aggressor side | (message index within the step << 1), step index t.
 * Env e's records go to trades[trade_off[e] + cursor ...], cursor = trade_cursor[e]
 * (or 0 when trade_cursor is NULL), in processing order over the steps of the call;
 * records beyond trade_off[e+1] are not written (counted as trade_overflow). */
typedef struct {
    int32_t *trades;          /* device [trade_off[n_envs]][8], or NULL (not recorded) */
    const int64_t *trade_off; /* device [n_envs+1], required when trades != NULL */
    int64_t *trade_cursor;    /* device [n_envs] in/out, or NULL */
    int32_t *n_trades;        /* device [n_steps][n_envs]: trades per env-step */
    int64_t *fills;           /* device [n_steps][n_agents][n_envs][4]: bought qty,
                                 bought notional, sold qty, sold notional */
    float *reward;            /* device [n_steps][n_agents][n_envs] */
    float *obs;               /* device [n_steps][n_agents][n_envs][40], or NULL */
    uint8_t *done;            /* device [n_steps][n_envs] */
    int32_t *actions;         /* device [n_steps][n_agents][n_envs]: actions taken, or NULL */
} lob_out;

/* Create a context (the environment configuration: book capacity of Table 2, agent types
 * of Sec. 4.1, order sizes and reward weights of Table 2 / Eq. 2-4): validates cfg,
 * allocates the books and per-env state on the current device.  Host-synchronous: it
 * allocates and uploads with blocking calls and launches no kernel, so it takes no
 * stream; the context is ready for any stream when it returns.  *out is NULL on failure.
 * Returns LOB_EINVAL / LOB_EUNSUPPORTED / LOB_ENOMEM / LOB_EHIP on failure. */
int lob_init(const lob_config *cfg, lob_ctx **out);

/* Start a new episode from a book state (Sec. 4, third paragraph: the book is initialised
 * from the state at the episode's start).  Loads every env's book from `snapshot`
 * (canonical layout, priority order, n <= cap; counts above an env's cap are clamped):
 * step 0, agents flat, the execution agent's task at exec_task, reference prices from
 * the best prices (the paper is silent on empty sides; reading: an empty side falls back
 * to one tick beyond the other side, 0 if both are empty).  Asynchronous on stream. */
int lob_reset(lob_ctx *ctx, const lob_books *snapshot, void *stream);

/* One env-step of every env, Sec. 4 steps 1-5 (action conversion with cancels, shuffle,
 * concatenation [cancels, orders, replay], book processing with trades recorded,
 * outcomes), in the plain per-step form: one launch, books loaded from and stored to
 * device memory.  Messages of step t = the context's step counter are
 * read from `msgs`.  actions: device int32 [n_agents][n_envs], or NULL for the uniform
 * random policy drawn in-kernel from the counter hash.  Out-of-range actions act as 0
 * (no quotes: every resting order of that agent is cancelled).  Outputs for 1 step.
 * LOB_ESTATE if not reset, the episode is over, or msgs has no row for this step. */
int lob_step(lob_ctx *ctx, const lob_msgs *msgs, const int32_t *actions, const lob_out *out,
             void *stream);

/* n_steps env-steps (Sec. 4 steps 1-5) of every env in one persistent launch per
 * capacity class (the batched form; the paper batches episodes by vectorising the step
 * over them, Sec. 4 and Fig. 1), books resident in LDS for all steps, envs pulled from a
 * work queue (longest first).
 * actions: device int32 [n_steps][n_agents][n_envs] or NULL (random policy).  Results
 * are identical to n_steps calls of lob_step. */
int lob_rollout(lob_ctx *ctx, const lob_msgs *msgs, int32_t n_steps, const int32_t *actions,
                const lob_out *out, void *stream);

/* Scheduling (this call, lob_schedule_get/set/balance, lob_set_padded and lob_autotune)
 * is the library's own: the paper is silent on it (it vectorises the step over
 * equal-shape episodes, Sec. 4 and Fig. 1).
 * Schedule plan for the next n_steps from the current step: orders each capacity
 * class's envs by decreasing message count (longest first), so that the envs that bound
 * the runtime start first; with several classes and a balance share set (the default,
 * see lob_schedule_balance), it also sizes each class's work queue.  Reads the CSR
 * offsets back to the host (synchronous: it first waits for this context's last launch,
 * or for the whole device once a launch of it was captured into a graph, so that no
 * launch still reading the previous plan's env list is running when it is rewritten).
 * Used by lob_step and lob_rollout until the next plan; results never depend on it. */
int lob_plan(lob_ctx *ctx, const lob_msgs *msgs, int32_t n_steps);

/* The launch schedule, one record of 5 int32 per capacity class (host array):
 * book records per side in LDS (the class's largest capacity), envs, waves (envs) per
 * workgroup, mode (0: one wave per env
 * dispatched by the hardware in plan order; 1: persistent workgroups pulling envs from a
 * device work queue), workgroups in mode 1 (0 = from occupancy).  Returns the number of
 * classes. */
int lob_schedule_get(const lob_ctx *ctx, int32_t *out, int32_t max_classes);

/* Set class k's schedule (waves 1, 2 or 4; mode 0 or 1; grid >= 0).  LOB_EUNSUPPORTED
 * if the workgroup would need more than 64 KiB of LDS.  Turns the balance share off
 * (lob_schedule_balance), so later plans keep the per-class schedules. */
int lob_schedule_set(lob_ctx *ctx, int32_t k, int32_t waves, int32_t mode, int32_t grid);

/* Schedule of several concurrent capacity classes.  permille in 1..1000: from the next
 * plan on, every class runs as a work queue (mode 1) whose workgroups hold a number of
 * envs proportional to the class's planned work (messages plus a fixed allowance per
 * env-step), all classes together sized to permille/1000 of the chip's LDS, so that the
 * classes finish together instead of the hardware dispatcher starving one of them
 * (default 880).  permille = 0: every class returns to its default schedule (mode 0)
 * and keeps whatever lob_schedule_set gives it.  A single class is never affected.
 * LOB_EINVAL outside 0..1000; results never depend on it. */
int lob_schedule_balance(lob_ctx *ctx, int32_t permille);

/* Batching ablation.  padded = 1 puts every env into one class whose LDS books are
 * sized for the largest capacity (uniform padding, the batching a map over envs of
 * equal shape gives); padded = 0 restores one class per book row count (the default).
 * Resets the plan and the schedules; results never depend on it.  Waits for this
 * context's launches as lob_plan does (host-synchronous); not callable during stream
 * capture. */
int lob_set_padded(lob_ctx *ctx, int32_t padded);

/* Autotuner: times schedules on the next n_steps of msgs from the current state
 * (restored after every run) and keeps the fastest.  One class: every (waves, mode) of
 * it.  Several classes (launched concurrently): the whole launch at balance shares 0,
 * 800 to 920 in steps of 20, and 960 permille (lob_schedule_balance), each run twice
 * and timed by its faster run.  Makes a plan first.
 * Synchronous; the buffers of `out` are overwritten (scratch).  Allocates and frees
 * temporary device memory for the state copy. */
int lob_autotune(lob_ctx *ctx, const lob_msgs *msgs, int32_t n_steps, const lob_out *out, void *stream);

/* Observation of the current state (Sec. 4 step 5; Sec. 4.1.1: statistics of the agent's
 * task such as its inventory; the 40 features are a reading), device float
 * [n_agents][n_envs][40], equal to the last step's observation (after reset the step
 * statistics are zero).  Asynchronous on stream. */
int lob_observe(lob_ctx *ctx, float *obs, void *stream);

/* Copy the books out in canonical layout: each side in price-time priority order
 * (Sec. 2.1), best first, unused slots zero.  Asynchronous on stream. */
int lob_export_books(lob_ctx *ctx, const lob_books *out, void *stream);

/* Copy the state out (device arrays), with lob_export_books everything an episode
 * continues from (lob_import_state; Sec. 4, third paragraph):
 *   env_state [n_envs][12]: last best bid, last best ask, mid2 (bid+ask) at the last step
 *     end, mid2 at reset, time of the last processed message (s, ns), steps since reset,
 *     mid2 change over the last step, then the last step's statistics (buyer- and
 *     seller-initiated volume, trades, last trade price);
 *   agent_state [n_envs][n_agents][6]: inventory, cash (ticks x shares), execution
 *     remaining, order-id counter, quantity bought and sold in the last step;
 *   counters [n_envs][11]: messages, trades, cancel and execution misses, evictions,
 *     evicted qty, drops, dropped qty, unfilled market qty, bad messages, trade records
 *     not written, ignored messages.
 * Any pointer may be NULL. */
int lob_export_state(lob_ctx *ctx, int64_t *env_state, int64_t *agent_state, int64_t *counters,
                     void *stream);

/* Continue every env from a given state (Sec. 4, third paragraph: an episode starts from
 * a book state; here any state exported by lob_export_books + lob_export_state, possibly
 * from another context or process, or edited): books in canonical layout (priority
 * order; counts clamped to each env's capacity), env_state / agent_state / counters in
 * the layouts of lob_export_state (device arrays; counters may be NULL = zero;
 * agent_state may be NULL only without agents).  `step` (0..episode_len) becomes the
 * step counter: the next step reads the messages of step `step` and is done at
 * episode_len; it replaces word 6 of every env's env_state.  The following steps then
 * give exactly what the exported context's following steps give.  Trade cursors are the
 * caller's.  Asynchronous on stream (the inputs must stay valid until it has run);
 * LOB_EINVAL for NULL books or state or a step out of range. */
int lob_import_state(lob_ctx *ctx, const lob_books *books, const int64_t *env_state, const int64_t *agent_state,
                     const int64_t *counters, int32_t step, void *stream);

/* ---- IPPO actor-critic (Sec. 4.2: independent PPO, separate weights per agent type) ----
 * Network per agent type: MLP 40 -> 256 -> 256 -> (9 policy logits + 1 value), tanh,
 * fp32 (the paper trains a recurrent network, Sec. 5.2.1; this feed-forward network is
 * the one the throughput workload fixes), flat parameters W1 [40][256] (input-major), b1 [256], W2 [256][256], b2 [256],
 * W3 [256][10], b3 [10]: LOB_PPO_PARAMS floats.  Products run on MFMA. */
#define LOB_PPO_PARAMS 78858

/* Policy forward for the rollout (Sec. 4.2: each agent type acts with its own network;
 * sampling by Gumbel-max is a reading, the paper is silent).  params: device [n_agents][LOB_PPO_PARAMS];
 * obs: device [n_agents][n][40], the env's observations as written; obs_scale: device
 * [40] or NULL, the policy's input scaling (feature c enters the network as obs * obs_scale[c];
 * the same argument of the PPO calls must match it); n_actions: host [n_agents] (1..9, the first n_actions
 * logits are the policy).  Samples one action per row by Gumbel-max with noise from the
 * counter hash of (seed', agent, action, t, row), seed' = seed + golden * (*epoch) when
 * epoch (a device uint64 counter, so that a captured graph draws new noise on each replay)
 * is given, else seed.  Outputs (device): logits [n_agents][n][10] (may be NULL), actions
 * [n_agents][n] int32, logp [n_agents][n] (log-probability of the sampled action), value
 * [n_agents][n].  Asynchronous on stream. */
int lob_policy_forward(const float *params, const float *obs, const float *obs_scale, int32_t n_agents, int32_t n,
                       const int32_t *n_actions,
                       uint64_t seed, const uint64_t *epoch, int32_t t, float *logits, int32_t *actions, float *logp,
                       float *value, void *stream);

/* Add one to a device uint64 counter (a kernel, so it can be captured in a graph; the
 * sampling epoch of lob_policy_forward).  Library plumbing, no passage of the paper. */
int lob_counter_bump(uint64_t *counter, void *stream);

/* Generalised advantage estimation over a rollout (the paper names IPPO, Sec. 4.2, and is
 * silent on the estimator; reading: GAE as in PPO, gamma and lambda from the caller, 0.99
 * and 0.95 in the IPPO workload), all arrays device [T][n] (column = env x agent): delta_t = r_t + gamma V_{t+1} (1 - d_t) - V_t with V_T = last_value [n],
 * A_t = delta_t + gamma lam (1 - d_t) A_{t+1}, ret = A + V.  done: uint8 (1 = the episode
 * ended at step t). */
int lob_gae(const float *reward, const float *value, const uint8_t *done, const float *last_value, int32_t T,
            int32_t n, float gamma, float lam, float *adv, float *ret, void *stream);

/* Bytes of device workspace lob_ppo_fwd_bwd needs for a minibatch of m samples
 * (LOB_EINVAL for m <= 0). */
int64_t lob_ppo_workspace_bytes(int32_t m);

/* Fused clipped-PPO loss and its gradient for one minibatch of one network (Sec. 4.2:
 * PPO per agent type; the clipped surrogate, value and entropy terms are PPO's, their
 * weights c_v, c_e the caller's since the paper is silent), with the activations
 * recomputed from obs (none stored between rollout and update; obs_scale as for
 * lob_policy_forward).  An action outside
 * [0, n_actions) counts as action 0, as the env step takes it.
 * obs [m][40], act [m] int32, logp_old, adv, ret, v_old [m] (device).  Loss =
 * policy + c_v value - c_e entropy with policy = -mean(min(r A, clip(r, 1-clip, 1+clip) A)),
 * r = exp(logp - logp_old), value = 0.5 mean(max((V-R)^2, (V_old + clip(V - V_old, -clip,
 * clip) - R)^2)), entropy = mean of the policy entropy.  Writes loss [4] = the sums over
 * the minibatch of the per-sample total, policy, value and entropy terms (divide by m for
 * the means) and grad [LOB_PPO_PARAMS] = gradient of the mean total loss (device).
 * workspace: device, 16-byte aligned, >= lob_ppo_workspace_bytes(m) (LOB_EINVAL otherwise);
 * params that are not 16-byte aligned are copied into it first, and W2 is written into it
 * transposed (both stream-ordered, before the fused kernel).
 * Deterministic: 256 workgroups each sum a fixed set of 64-sample tiles in order, and
 * their partials are summed in a fixed order. */
int lob_ppo_fwd_bwd(const float *params, const float *obs, const float *obs_scale, const int32_t *act,
                    const float *logp_old,
                    const float *adv, const float *ret, const float *v_old, int32_t m, int32_t n_actions, float clip,
                    float c_v, float c_e, float *workspace, int64_t workspace_bytes, float *loss, float *grad,
                    void *stream);

/* lob_ppo_fwd_bwd without a workspace argument, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight training loops, harnesses that forbid
 * allocation).  The workspace is a fixed array in device memory that the library holds on
 * every GPU it runs on until the process ends: PPO_SCRATCH = 256 workgroup partials of
 * 78,864 floats, 4 chunk sums of the first reduction level, room for an aligned
 * parameter copy and for W2 transposed (256 x 256 floats), 82,596,168 bytes (about
 * 83 MB); m is not limited by it, since the
 * partials do not grow with m (LOB_EINVAL if a minibatch ever needed more).  Allocates
 * nothing and calls no allocating routine; the array's device address is resolved once
 * per GPU on the first call there.  Same arguments, results (bit for bit) and errors as
 * lob_ppo_fwd_bwd otherwise.  Every call on one GPU uses that GPU's one array: calls that
 * overlap on one GPU (other streams, other threads) race and must be ordered by the
 * caller; nothing in the array needs clearing between calls (each call writes every
 * partial it reads). */
int lob_ppo_fwd_bwd_noalloc(const float *params, const float *obs, const float *obs_scale, const int32_t *act,
                            const float *logp_old,
                            const float *adv, const float *ret, const float *v_old, int32_t m, int32_t n_actions,
                            float clip, float c_v, float c_e, float *loss, float *grad, void *stream);

/* ---- Recurrent actor-critic (Sec. 5.2.1: the agents' networks are GRU-based; one per
 * agent type, Sec. 4.2).  The paper gives no sizes; reading: e_t = tanh(x_t W_e + b_e)
 * (40 -> 128), a gated recurrent unit of 128 (gates r, u, n: r = sigmoid(e W_ir + b_ir +
 * h W_hr + b_hr), u likewise, n = tanh(e W_in + b_in + r (h W_hn + b_hn)), h' = (1 - u) n
 * + u h), out_t = h_t W_o + b_o (9 logits + value); the hidden state is zeroed at an
 * episode's first step.  Flat fp32 parameters: W_e [40][128], b_e [128], W_i [128][384]
 * (gate columns r | u | n), b_i [384], W_h [128][384], b_h [384], W_o [128][10], b_o [10]:
 * LOB_GRU_PARAMS floats.  Products run on MFMA. */
#define LOB_GRU_PARAMS 105610
#define LOB_GRU_HIDDEN 128

/* One rollout step of the recurrent policy for every agent: params [n_agents][params],
 * obs [n_agents][n][40] (obs_scale as for lob_policy_forward), h_in / h_out [n_agents][n][128] (device; h_out may be h_in),
 * start [n] uint8 (device, 1 = the episode starts at this step: h_in is taken as zero) or
 * NULL.  Samples as lob_policy_forward (same counter hash and epoch; logits may be NULL).
 * Asynchronous on stream. */
int lob_gru_step(const float *params, const float *obs, const float *obs_scale, const float *h_in, float *h_out,
                 const uint8_t *start,
                 int32_t n_agents, int32_t n, const int32_t *n_actions, uint64_t seed, const uint64_t *epoch, int32_t t,
                 float *logits, int32_t *actions, float *logp, float *value, void *stream);

/* Bytes of device workspace lob_gru_ppo_fwd_bwd needs for m sequences of T steps
 * (LOB_EINVAL for T or m <= 0): the hidden states, the per-sample embedding, input-gate
 * products (then their gradients), hidden-gate gradients, embedding and output gradients
 * (1,168 floats per sample), loss sums per 64 samples, the prepared weights and the
 * weight-gradient partials. */
int64_t lob_gru_ppo_workspace_bytes(int32_t T, int32_t m);

/* The clipped-PPO loss (the same per-sample terms as lob_ppo_fwd_bwd, averaged over the T
 * m samples) of one network over a minibatch of m whole sequences, and its gradient
 * through time.  obs [T][m][40] (obs_scale as for lob_policy_forward), start [T][m] uint8, h0 [m][128] (the state before step
 * 0), act, logp_old, adv, ret, v_old [T][m] (device).  The products that do not depend on
 * the previous state (embedding, input gates, outputs and loss terms, embedding gradient,
 * weight gradients) run batched over all samples; the forward recurrence keeps only the
 * hidden states and the backward one recomputes each step's hidden-gate products.
 * Writes loss [4] (sums over the samples of the total, policy, value and entropy terms)
 * and grad [LOB_GRU_PARAMS] (gradient of the mean total loss).  workspace: device,
 * 16-byte aligned, >= lob_gru_ppo_workspace_bytes(T, m) (LOB_EINVAL otherwise).
 * Deterministic (fixed tiles and summation orders).  An action outside [0, n_actions)
 * counts as action 0. */
int lob_gru_ppo_fwd_bwd(const float *params, const float *obs, const float *obs_scale, const uint8_t *start,
                        const float *h0,
                        const int32_t *act, const float *logp_old, const float *adv, const float *ret,
                        const float *v_old, int32_t T, int32_t m, int32_t n_actions, float clip, float c_v, float c_e,
                        float *workspace, int64_t workspace_bytes, float *loss, float *grad, void *stream);

/* Steps taken since the last reset or import (host-side counter; library plumbing). */
int lob_current_step(const lob_ctx *ctx);

/* Free the context (synchronises the device first).  NULL is a no-op.  Library plumbing. */
int lob_destroy(lob_ctx *ctx);

/* Static message for an error code (library plumbing). */
const char *lob_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif
