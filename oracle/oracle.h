/*
 * CPU oracle for the batched limit-order-book environment step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load this library.  The product path (the HIP library) shares
 * no code, header, table or helper with it.
 *
 * The oracle is a plain sequential implementation written from the paper:
 *   - price-time-priority continuous double auction (Sec. 2.1);
 *   - the five-stage environment step (Sec. 4, numbered step list): action conversion
 *     with cancels unless re-quoted at the same level, random shuffle of the agents'
 *     messages, concatenation [cancels, actions, replay] in that order, processing by
 *     the order book with trades recorded, and step outcomes;
 *   - the agent types of Sec. 4.1 (execution, market making with the fixed-quantity
 *     action space, directional trading);
 *   - rewards from Eq. 2 (slippage), Eq. 3 (Spooner) and Eq. 4 (buy-sell).
 * Where the paper is silent, the reading used is documented next to the code.
 *
 * All arrays are host memory owned by the caller.  Layouts match the GPU library's
 * documented layouts so that outputs compare element by element.
 */
#ifndef LOB_ORACLE_H
#define LOB_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t n_envs;
    int32_t n_agents;         /* 0..4 */
    int32_t max_cap;          /* stride of the book arrays */
    int32_t episode_len;
    const int32_t *cap;       /* [n_envs] per-side capacity, 1..max_cap */
    const int32_t *agent_kind;/* [n_agents] 0 execution, 1 market maker (fixed quantity), 2 directional,
                                 3 market maker rewarded by Eq. 4, 4 market maker (spread-skew),
                                 5 market maker (AvSt), 6 TWAP execution baseline, 7 Avellaneda-Stoikov
                                 market-making baseline */
    uint64_t seed;
    int32_t exec_task;        /* shares the execution agent sells per episode */
    int32_t exec_q0;          /* execution order quantity */
    int32_t mm_q;             /* market-maker quote quantity */
    int32_t dir_q;            /* directional order quantity */
    float exec_penalty;       /* end-of-episode penalty per unfilled share (times P_init) */
    float mm_lambda;          /* Spooner weighting of positive inventory PnL */
    float mm_rho;             /* quadratic inventory penalty factor */
    float pad_;
    const int32_t *env_id;    /* [n_envs] env index used in the hash keys, or NULL (= position) */
    float avst_gamma;         /* Avellaneda-Stoikov quotes: base risk aversion (> 0) */
    float avst_sigma2;        /* price variance per step, ticks^2 (>= 0) */
    float avst_kappa;         /* order-arrival decay per tick (> 0) */
    float pad2_;
} or_config;

/* ---- single book (unit tests) ---- */
void *ob_new(int32_t cap);
void ob_free(void *b);
/* Process one message {ts, price, qty, oid, tid, tsec, tns}; trade records (8 int32
 * each) are appended to trades up to max_trades; counters[10] accumulate.  Returns
 * the number of trades produced (also those not written). */
int32_t ob_process(void *b, const int32_t *msg, int32_t seq, int32_t t, int32_t *trades,
                   int32_t max_trades, int64_t *counters);
/* Export one side (0 bids, 1 asks) in priority order as [n][6] records. */
int32_t ob_export(void *b, int32_t side, int32_t *out, int32_t max_n);
/* Replace one side by n records [n][6] given in priority order. */
void ob_load(void *b, int32_t side, const int32_t *in, int32_t n);

/* ---- environments ---- */
void *oe_new(const or_config *cfg);
void oe_free(void *o);
int32_t oe_reset(void *o, const int32_t *price, const int32_t *qty, const int32_t *oid,
                 const int32_t *tid, const int32_t *tsec, const int32_t *tns, const int32_t *n);
int32_t oe_step(void *o, int32_t n_steps,
                const int32_t *ts, const int32_t *price, const int32_t *qty, const int32_t *oid,
                const int32_t *tid, const int32_t *tsec, const int32_t *tns,
                const int64_t *off, int32_t off_steps,
                const int32_t *actions,
                int32_t *trades, const int64_t *trade_off, int32_t *n_trades,
                int64_t *fills, float *reward, float *obs, uint8_t *done, int32_t *actions_out,
                int32_t n_threads);
int32_t oe_observe(void *o, float *obs);
int32_t oe_export_books(void *o, int32_t *price, int32_t *qty, int32_t *oid, int32_t *tid,
                        int32_t *tsec, int32_t *tns, int32_t *n);
/* env_state [n_envs][12], agent_state [n_envs][n_agents][6], counters [n_envs][11]. */
int32_t oe_export_state(void *o, int64_t *env_state, int64_t *agent_state, int64_t *counters);
/* Continue every env from the given books and state (the exported layouts); every env's
 * step counter becomes `step`; counters may be NULL (zero). */
int32_t oe_import_state(void *o, const int32_t *price, const int32_t *qty, const int32_t *oid,
                        const int32_t *tid, const int32_t *tsec, const int32_t *tns, const int32_t *n,
                        const int64_t *env_state, const int64_t *agent_state, const int64_t *counters,
                        int32_t step);

/* The method's counter hash (SplitMix64 output function applied in a chain). */
uint64_t oe_hash(uint64_t seed, uint64_t dom, uint64_t a, uint64_t b, uint64_t c);
/* One application of the SplitMix64 output function (state increment included). */
uint64_t oe_mix(uint64_t z);

#ifdef __cplusplus
}
#endif
#endif
