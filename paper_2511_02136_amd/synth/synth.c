/*
 * Seeded synthetic market-by-order (MBO) stream generator.
 *
 * This module produces INPUTS only: message streams in structure-of-arrays form,
 * CSR step offsets, per-env book capacities and a reset snapshot per env.  It holds
 * none of the order-book method's arithmetic (no matching, no priority rules beyond
 * laying out the initial snapshot in price order, which is what a market-data
 * snapshot file holds).  Both the CPU oracle and the GPU path consume its output.
 *
 * The paper replays LOBSTER messages (Sec. 4, third paragraph: the whole dataset is
 * stored contiguously and episodes are indexed at run time).  That data is not
 * available, so this generator stands in for it with the shapes and mixes of the
 * benchmark workloads:
 *   - message mix: 50% limit, 20% partial cancel, 20% delete, 10% market;
 *   - mid price: a random walk in ticks (+-1 with probability 0.05 each per message);
 *   - limit price: mid -/+ g ticks, g ~ Geometric(p = 0.3) counted as failures, capped;
 *   - size: lognormal(mu = 4, sigma = 1) rounded to >= 1, via a 4096-entry quantile table;
 *   - cancels target one of the last 256 limit orders issued in that env;
 *   - time advances 1..1000 ns per message.
 *
 * Every draw comes from a counter-based hash keyed by (seed, env, step, msg, field),
 * so any env regenerates identically on its own and envs generate in parallel.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SYN_LIMIT 1
#define SYN_PCANCEL 2
#define SYN_DELETE 3
#define SYN_MARKET 4
#define SYN_EXECUTE 5
#define SYN_IGNORED 6

typedef struct {
    int32_t n_envs;
    int32_t n_steps;
    int32_t msgs_per_step;       /* > 0: fixed count per step */
    int32_t msgs_lo, msgs_hi;    /* msgs_per_step == 0: per-env count uniform in [lo, hi] */
    int32_t burst_pct;           /* percent of steps that are bursts (0 = none) */
    int32_t burst_extra;         /* extra cancel messages appended in a burst step */
    int32_t cap_fixed;           /* > 0: every env has this per-side capacity */
    int32_t n_cap_choices;       /* cap_fixed == 0: per-env capacity uniform over these */
    int32_t cap_choices[8];
    int32_t mid0;                /* initial mid price in ticks */
    int32_t snapshot_fill_pct;   /* percent of cap placed per side in the reset snapshot */
    int32_t exec_pct;            /* percent of messages turned into replayed executions */
    int32_t ignored_pct;         /* percent turned into messages the book ignores */
    uint64_t seed;
} synth_config;

/* ---- counter hash: SplitMix64 output function (Steele, Lea, Flood 2014) ---- */
static inline uint64_t syn_mix(uint64_t z) {
    z += 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* field tags (domain separation between draws of one message) */
enum {
    F_TYPE = 1, F_SIDE, F_SIZE, F_MID, F_CANCEL, F_PQTY, F_TIME, F_BURSTTYPE,
    F_GEOM0 = 64,          /* F_GEOM0 + k: k-th geometric trial */
    F_ENVCAP = 1001, F_ENVMSGS, F_BURST,
    F_XTYPE = 2001, F_XAGENT, F_XAGENTK
};

static inline uint64_t syn_base(uint64_t seed, uint64_t e, uint64_t t, uint64_t m) {
    return syn_mix(syn_mix(syn_mix(syn_mix(seed) ^ e) ^ t) ^ m);
}
static inline uint32_t syn_u32(uint64_t base, uint64_t field) {
    return (uint32_t)(syn_mix(base ^ (field * 0xD1B54A32D192ED03ULL)) >> 32);
}

/* ---- lognormal(4, 1) size table ---- */
static int32_t g_size_table[4096];
static pthread_once_t g_size_once = PTHREAD_ONCE_INIT;

/* Standard normal quantile: Acklam's rational approximation refined by one Halley
 * step on erfc (rel. error far below the table's resolution). */
static double syn_norm_quantile(double p) {
    static const double a[6] = {-3.969683028665376e+01, 2.209460984245205e+02,
                                -2.759285104469687e+02, 1.383577518672690e+02,
                                -3.066479806614716e+01, 2.506628277459239e+00};
    static const double b[5] = {-5.447609879822406e+01, 1.615858368580409e+02,
                                -1.556989798598866e+02, 6.680131188771972e+01,
                                -1.328068155288572e+01};
    static const double c[6] = {-7.784894002430293e-03, -3.223964580411365e-01,
                                -2.400758277161838e+00, -2.549732539343734e+00,
                                4.374664141464968e+00, 2.938163982698783e+00};
    static const double d[4] = {7.784695709041462e-03, 3.224671290700398e-01,
                                2.445134137142996e+00, 3.754408661907416e+00};
    double q, r, x;
    if (p < 0.02425) {
        q = sqrt(-2 * log(p));
        x = (((((c[0] * q + c[1]) * q + c[2]) * q + c[3]) * q + c[4]) * q + c[5]) /
            ((((d[0] * q + d[1]) * q + d[2]) * q + d[3]) * q + 1);
    } else if (p <= 1 - 0.02425) {
        q = p - 0.5;
        r = q * q;
        x = (((((a[0] * r + a[1]) * r + a[2]) * r + a[3]) * r + a[4]) * r + a[5]) * q /
            (((((b[0] * r + b[1]) * r + b[2]) * r + b[3]) * r + b[4]) * r + 1);
    } else {
        q = sqrt(-2 * log(1 - p));
        x = -(((((c[0] * q + c[1]) * q + c[2]) * q + c[3]) * q + c[4]) * q + c[5]) /
            ((((d[0] * q + d[1]) * q + d[2]) * q + d[3]) * q + 1);
    }
    double err = 0.5 * erfc(-x / sqrt(2.0)) - p;
    double u = err * sqrt(2 * M_PI) * exp(x * x / 2);
    return x - u / (1 + x * u / 2);
}

static void syn_build_size_table(void) {
    for (int i = 0; i < 4096; ++i) {
        double u = (i + 0.5) / 4096.0;
        double x = exp(4.0 + 1.0 * syn_norm_quantile(u));
        double q = floor(x + 0.5);
        if (q < 1) q = 1;
        if (q > 1e9) q = 1e9;
        g_size_table[i] = (int32_t)q;
    }
}

static inline int32_t syn_size(uint64_t base, uint64_t field) {
    return g_size_table[syn_u32(base, field) >> 20];
}

static inline int32_t syn_geom(uint64_t base) {
    const uint32_t thr = 3006477107u; /* floor(0.7 * 2^32): a trial fails with p = 0.7 */
    int32_t k = 0;
    while (k < 255 && syn_u32(base, F_GEOM0 + k) < thr) ++k;
    return k;
}

/* ---- per-env shape ---- */
int32_t synth_env_cap(const synth_config *c, int32_t e) {
    if (c->cap_fixed > 0) return c->cap_fixed;
    uint64_t b = syn_base(c->seed, (uint64_t)e, 0xFFFFFFFFull, 0);
    return c->cap_choices[syn_u32(b, F_ENVCAP) % (uint32_t)c->n_cap_choices];
}

static int32_t syn_env_base_msgs(const synth_config *c, int32_t e) {
    if (c->msgs_per_step > 0) return c->msgs_per_step;
    uint64_t b = syn_base(c->seed, (uint64_t)e, 0xFFFFFFFFull, 0);
    return c->msgs_lo + (int32_t)(syn_u32(b, F_ENVMSGS) % (uint32_t)(c->msgs_hi - c->msgs_lo + 1));
}

static int syn_is_burst(const synth_config *c, int32_t e, int32_t t) {
    if (c->burst_pct <= 0) return 0;
    uint64_t b = syn_base(c->seed, (uint64_t)e, (uint64_t)t, 0xFFFFFFFFull);
    return (int)(syn_u32(b, F_BURST) % 100u) < c->burst_pct;
}

int32_t synth_step_count(const synth_config *c, int32_t e, int32_t t) {
    int32_t n = syn_env_base_msgs(c, e);
    if (syn_is_burst(c, e, t)) n += c->burst_extra;
    return n;
}

/* CSR offsets: off[e*(n_steps+1) + t] = index of env e's first message of step t;
 * env-major, so env e's messages are contiguous and off[e][n_steps] == off[e+1][0].
 * Returns the total message count. */
int64_t synth_offsets(const synth_config *c, int64_t *off) {
    int64_t pos = 0;
    for (int32_t e = 0; e < c->n_envs; ++e) {
        int64_t *row = off + (int64_t)e * (c->n_steps + 1);
        for (int32_t t = 0; t < c->n_steps; ++t) {
            row[t] = pos;
            pos += synth_step_count(c, e, t);
        }
        row[c->n_steps] = pos;
    }
    return pos;
}

typedef struct {
    int32_t *ts, *price, *qty, *oid, *tid, *tsec, *tns;
} syn_msgs;

typedef struct {
    /* [n_envs][2][max_cap] each, side 0 = bids (best first), side 1 = asks */
    int32_t *price, *qty, *oid, *tid, *tsec, *tns;
    int32_t *n; /* [n_envs][2] */
} syn_books;

typedef struct {
    int32_t oid, side, price, qty;
} syn_ring_entry;

typedef struct {
    const synth_config *c;
    const int64_t *off;
    int32_t max_cap;
    syn_msgs m;
    syn_books b;
    int32_t e0, e1;
} syn_job;

static void syn_env(const synth_config *c, int32_t e, const int64_t *off, int32_t max_cap,
                    const syn_msgs *m, const syn_books *bk) {
    syn_ring_entry ring[256];
    int32_t ring_n = 0, ring_head = 0;
    int32_t mid = c->mid0;
    int32_t next_oid = 1;
    int32_t tsec = 34200, tns = 0; /* 09:30:00 */
    const int32_t cap = synth_env_cap(c, e);

    /* ---- reset snapshot: fill_pct% of cap per side, bids at mid-1-g, asks at mid+1+g,
     * arrival order bid, ask, bid, ask, ...; laid out best price first, arrival order
     * within a price (the order of a market-data snapshot). ---- */
    int32_t per_side = (int32_t)(((int64_t)cap * c->snapshot_fill_pct) / 100);
    if (per_side < 1) per_side = 1;
    if (per_side > cap) per_side = cap;
    for (int side = 0; side < 2; ++side) bk->n[e * 2 + side] = 0;
    for (int32_t j = 0; j < 2 * per_side; ++j) {
        uint64_t base = syn_base(c->seed, (uint64_t)e, 0xFFFFFFFEull, (uint64_t)j);
        int side = j & 1;
        int32_t g = syn_geom(base);
        int32_t price = side == 0 ? mid - 1 - g : mid + 1 + g;
        int32_t qty = syn_size(base, F_SIZE);
        int32_t oid = next_oid++;
        tns += 1 + (int32_t)(syn_u32(base, F_TIME) % 1000u);
        if (tns >= 1000000000) { tns -= 1000000000; ++tsec; }
        /* insertion into the price-ordered snapshot list (after equal prices) */
        int64_t sbase = ((int64_t)e * 2 + side) * max_cap;
        int32_t n = bk->n[e * 2 + side];
        int32_t pos = n;
        while (pos > 0) {
            int32_t pp = bk->price[sbase + pos - 1];
            int better = side == 0 ? (pp < price) : (pp > price);
            if (!better) break;
            --pos;
        }
        for (int32_t s = n; s > pos; --s) {
            bk->price[sbase + s] = bk->price[sbase + s - 1];
            bk->qty[sbase + s] = bk->qty[sbase + s - 1];
            bk->oid[sbase + s] = bk->oid[sbase + s - 1];
            bk->tid[sbase + s] = bk->tid[sbase + s - 1];
            bk->tsec[sbase + s] = bk->tsec[sbase + s - 1];
            bk->tns[sbase + s] = bk->tns[sbase + s - 1];
        }
        bk->price[sbase + pos] = price;
        bk->qty[sbase + pos] = qty;
        bk->oid[sbase + pos] = oid;
        bk->tid[sbase + pos] = 0;
        bk->tsec[sbase + pos] = tsec;
        bk->tns[sbase + pos] = tns;
        bk->n[e * 2 + side] = n + 1;
        ring[ring_head & 255] = (syn_ring_entry){oid, side, price, qty};
        ++ring_head;
        if (ring_n < 256) ++ring_n;
    }
    for (int side = 0; side < 2; ++side) {
        int64_t sbase = ((int64_t)e * 2 + side) * max_cap;
        for (int32_t s = bk->n[e * 2 + side]; s < max_cap; ++s) {
            bk->price[sbase + s] = 0; bk->qty[sbase + s] = 0; bk->oid[sbase + s] = 0;
            bk->tid[sbase + s] = 0; bk->tsec[sbase + s] = 0; bk->tns[sbase + s] = 0;
        }
    }

    /* ---- the message stream ---- */
    const int64_t *row = off + (int64_t)e * (c->n_steps + 1);
    const int32_t base_n = syn_env_base_msgs(c, e);
    for (int32_t t = 0; t < c->n_steps; ++t) {
        int64_t i0 = row[t], i1 = row[t + 1];
        for (int64_t i = i0; i < i1; ++i) {
            int32_t mi = (int32_t)(i - i0);
            uint64_t base = syn_base(c->seed, (uint64_t)e, (uint64_t)t, (uint64_t)mi);
            uint32_t um = syn_u32(base, F_MID) % 100u;
            if (um < 5) --mid; else if (um < 10) ++mid;
            int32_t type;
            if (mi >= base_n) {
                type = (syn_u32(base, F_BURSTTYPE) & 1u) ? SYN_DELETE : SYN_PCANCEL;
            } else {
                uint32_t ut = syn_u32(base, F_TYPE) % 100u;
                type = ut < 50 ? SYN_LIMIT : ut < 70 ? SYN_PCANCEL : ut < 90 ? SYN_DELETE : SYN_MARKET;
                if (c->exec_pct > 0 || c->ignored_pct > 0) {
                    /* (draws that exist only in workloads using these types) */
                    uint32_t ux = syn_u32(base, F_XTYPE) % 100u;
                    if (ux < (uint32_t)c->exec_pct) type = SYN_EXECUTE;
                    else if (ux < (uint32_t)(c->exec_pct + c->ignored_pct)) type = SYN_IGNORED;
                }
            }
            int32_t side = (int32_t)(syn_u32(base, F_SIDE) & 1u);
            int32_t price = 0, qty = 0, oid = 0;
            if (type == SYN_LIMIT) {
                int32_t g = syn_geom(base);
                price = side == 0 ? mid - g : mid + g;
                qty = syn_size(base, F_SIZE);
                oid = next_oid++;
                ring[ring_head & 255] = (syn_ring_entry){oid, side, price, qty};
                ++ring_head;
                if (ring_n < 256) ++ring_n;
            } else if (type == SYN_MARKET) {
                qty = syn_size(base, F_SIZE);
                oid = next_oid++;
                price = mid;
            } else if (type == SYN_IGNORED) {
                qty = syn_size(base, F_SIZE);
                price = mid;
            } else if (type == SYN_EXECUTE && (syn_u32(base, F_XAGENT) & 3u) == 0) {
                /* an execution naming one of the first 64 orders of agent 0 or 1 (agent
                 * order ids are 2^30 | agent << 26 | counter), resting or not */
                uint32_t ua = syn_u32(base, F_XAGENTK);
                oid = (int32_t)((1u << 30) | ((ua & 1u) << 26) | ((ua >> 1) & 63u));
                qty = syn_size(base, F_SIZE);
                price = mid;
            } else {
                if (ring_n > 0) {
                    uint32_t k = syn_u32(base, F_CANCEL) % (uint32_t)ring_n;
                    syn_ring_entry r = ring[(ring_head - 1 - (int32_t)k) & 255];
                    side = r.side; price = r.price; oid = r.oid;
                    /* partial cancels, and half of the executions, take part of the order */
                    const int part = type == SYN_PCANCEL || (type == SYN_EXECUTE && (syn_u32(base, F_XAGENT) & 4u));
                    qty = part ? 1 + (int32_t)(syn_u32(base, F_PQTY) % (uint32_t)r.qty) : r.qty;
                } else {
                    oid = 0; qty = 1;
                }
            }
            tns += 1 + (int32_t)(syn_u32(base, F_TIME) % 1000u);
            if (tns >= 1000000000) { tns -= 1000000000; ++tsec; }
            m->ts[i] = type | (side << 8);
            m->price[i] = price;
            m->qty[i] = qty;
            m->oid[i] = oid;
            m->tid[i] = 0;
            m->tsec[i] = tsec;
            m->tns[i] = tns;
        }
    }
}

static void *syn_worker(void *arg) {
    syn_job *j = (syn_job *)arg;
    for (int32_t e = j->e0; e < j->e1; ++e) syn_env(j->c, e, j->off, j->max_cap, &j->m, &j->b);
    return NULL;
}

/* Generate the reset snapshots and the message stream of every env.
 * off must come from synth_offsets(); message arrays have off[n_envs*(n_steps+1)-1]
 * entries; book arrays are [n_envs][2][max_cap] with max_cap >= every env's cap. */
int synth_generate(const synth_config *c, const int64_t *off, int32_t max_cap,
                   int32_t *ts, int32_t *price, int32_t *qty, int32_t *oid, int32_t *tid,
                   int32_t *tsec, int32_t *tns,
                   int32_t *b_price, int32_t *b_qty, int32_t *b_oid, int32_t *b_tid,
                   int32_t *b_tsec, int32_t *b_tns, int32_t *b_n, int32_t n_threads) {
    pthread_once(&g_size_once, syn_build_size_table);
    if (c->n_envs <= 0 || c->n_steps < 0) return -1;
    for (int32_t e = 0; e < c->n_envs; ++e)
        if (synth_env_cap(c, e) > max_cap) return -1;
    if (n_threads < 1) n_threads = 1;
    if (n_threads > c->n_envs) n_threads = c->n_envs;
    syn_msgs m = {ts, price, qty, oid, tid, tsec, tns};
    syn_books b = {b_price, b_qty, b_oid, b_tid, b_tsec, b_tns, b_n};
    syn_job *jobs = (syn_job *)calloc((size_t)n_threads, sizeof(syn_job));
    pthread_t *th = (pthread_t *)calloc((size_t)n_threads, sizeof(pthread_t));
    for (int32_t k = 0; k < n_threads; ++k) {
        jobs[k].c = c; jobs[k].off = off; jobs[k].max_cap = max_cap; jobs[k].m = m; jobs[k].b = b;
        jobs[k].e0 = (int32_t)((int64_t)c->n_envs * k / n_threads);
        jobs[k].e1 = (int32_t)((int64_t)c->n_envs * (k + 1) / n_threads);
        pthread_create(&th[k], NULL, syn_worker, &jobs[k]);
    }
    for (int32_t k = 0; k < n_threads; ++k) pthread_join(th[k], NULL);
    free(jobs);
    free(th);
    return 0;
}

/* The size table (for distribution tests). */
void synth_size_table(int32_t *out) {
    pthread_once(&g_size_once, syn_build_size_table);
    memcpy(out, g_size_table, sizeof(g_size_table));
}

/* Raw counter hash (for tests of the generator's statistics). */
uint32_t synth_u32(uint64_t seed, uint64_t e, uint64_t t, uint64_t m, uint64_t field) {
    return syn_u32(syn_base(seed, e, t, m), field);
}
