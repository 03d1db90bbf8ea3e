/*
 * Batched limit-order-book environment step: HIP kernels for gfx950 and the C-ABI.
 *
 * The step is the five-stage env step of JaxMARL-HFT (arXiv 2511.02136, Sec. 4):
 * action conversion with cancels (step 1), shuffle (step 2), concatenation with the
 * replayed messages (step 3), price-time-priority matching with trades recorded (step 4,
 * Sec. 2.1), and outcomes (step 5: fills, rewards by Eq. 2-4, observations).
 *
 * Design (MI355X-first):
 *   - one wavefront per environment; the book of both sides is LDS-resident, one
 *     16-byte record per order (price|qty, oid|tid) and a 4-byte reference to its time
 *     (the time itself stays in the message stream or in the book as loaded, and is
 *     looked up when the books are stored), ordered from the worst order to the best so
 *     the top of the book is the end of the live range; record j is handled by lane
 *     j%64 of row j/64 (see lob_device.h);
 *   - a book message is a few wave-wide LDS instructions: a ballot search from the top
 *     row down for cancels and for the insertion rank, a one-pass shift of the rows an
 *     insertion or removal touches (usually one), and matching on the 64 best orders at
 *     once (a prefix sum of their quantities finds the fill point; fills of the best
 *     order move nothing);
 *   - agent orders and replayed messages run through one loop, 64 messages per chunk
 *     staged with coalesced SoA loads;
 *   - per step, the agents' desired levels and their resting orders (collected in one
 *     pass per side) are held in registers, lane-parallel, and their observation
 *     features are formed one per lane; state that only accumulates (the mid-price run
 *     sums) is kept in vector registers, so that the CU's one scalar unit, which issues
 *     most of a message's instructions, carries only what steers control flow;
 *   - envs are grouped by capacity class (books spanning the same number of rows), each
 *     class's launch sized in LDS for its largest capacity; the persistent form keeps
 *     books in LDS for all steps of a rollout and pulls envs from a device work queue,
 *     longest first.
 *
 * Floating point: rewards are evaluated in double in a fixed order with contraction
 * disabled and rounded once to float; observation features are exact integers rounded
 * to float.
 */
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "lob.h"
#include "lob_device.h"

#pragma clang fp contract(off)

namespace lobk {

constexpr int MAXA = LOB_MAX_AGENTS;
constexpr int FIND_ROWS = 4; /* rows an order-id search loads per LDS round trip */

/* agent kinds by role: execution tasks (a sell task with a remainder), market makers
 * rewarded by Eq. 3 (Spooner) */
__host__ __device__ constexpr bool exec_kind(int k) { return k == LOB_AGENT_EXEC || k == LOB_AGENT_EXEC_TWAP; }
__host__ __device__ constexpr bool spooner_kind(int k) {
    return k == LOB_AGENT_MM || k == LOB_AGENT_MM_SPREADSKEW || k == LOB_AGENT_MM_AVST || k == LOB_AGENT_MM_AS;
}
/* actions of each kind (the baselines take none: one action, not used) */
__host__ __device__ constexpr int kind_actions(int k) {
    return k == LOB_AGENT_DIR ? 3 : ((k == LOB_AGENT_EXEC_TWAP || k == LOB_AGENT_MM_AS) ? 1 : 9);
}
/* floor(x / 2) for any sign */
__device__ __forceinline__ int64_t floor_div2(int64_t x) { return x >= 0 ? x / 2 : -((-x + 1) / 2); }
/* a price from a double quote, limited to +-2^30 */
__device__ __forceinline__ int quote_price(double x) {
    const double lim = 1073741824.0;
    return (int)(x < -lim ? -lim : (x > lim ? lim : x));
}
constexpr int MAXLV = 8;          /* desired price levels per agent per step */
constexpr int AGW = 8;            /* internal agent words: inv, cash, rem, ctr, step_bq, step_sq */
constexpr int STW = 4;            /* step statistics: buy vol, sell vol, trades, last price */
constexpr int ENVW = 8;           /* internal env state words (the exported state adds the STW statistics) */
static_assert(ENVW + STW == LOB_ENV_STATE_WORDS, "exported env state = internal env state + step statistics");
static_assert(LOB_AGENT_STATE_WORDS <= AGW, "exported agent words");

/* Per-wave LDS layout after the book (int32 word offsets), for A agents (at most 8 new
 * orders per agent per step):
 *   act  8A x 8: new orders of the step (ts, price, qty, oid, tid, time reference, -, -)
 *   perm 8A: shuffled order
 *   ag   int64 A x AGW: agent state  fl   int64 A x 4: fills of the step
 *   obk  int64 22 + 3A: depth buckets, totals, own stats (shares act's words: the
 *        observation is built after the messages, the new orders before them)
 *   env  int64 8  st  int64 STW */
struct XL {
    int act, perm, ag, fl, obk, env, st, words;
};
__host__ __device__ constexpr XL x_layout(int A) {
    XL x{};
    x.act = 0;
    x.perm = x.act + 8 * A * 8;
    x.ag = (x.perm + 8 * A + 1) & ~1;
    x.fl = x.ag + A * AGW * 2;
    x.obk = x.act;
    x.env = x.fl + A * 4 * 2;
    x.st = x.env + 8 * 2;
    x.words = x.st + STW * 2;
    return x;
}
static_assert(x_layout(MAXA).words < 1024, "extra LDS");
static_assert((22 + 3 * 1) * 2 <= 8 * 1 * 8, "observation accumulators fit in the new-order block");

/* per side and order: a record of 4 words (price, qty, oid, tid) and a time reference;
 * rounded to 16 bytes so that every wave's records are 16-byte aligned (one 128-bit LDS
 * access per record, conflict-free across a row) */
__host__ __device__ constexpr int lds_words_for(int capp, int n_agents) {
    return (10 * capp + x_layout(n_agents).words + 3) & ~3;
}

constexpr int REC = 2; /* int2 pairs per book record: (price, qty), (oid, tid) */
/* time references: >= 0 an index into the env's message stream (relative to its first
 * message); TREF_LOADED | i slot i of the side as loaded at the launch's start (the
 * time is in the books in memory); TREF_START the last processed time at the launch's
 * start */
constexpr int TREF_LOADED = (int)0x80000000u, TREF_START = (int)0xC0000000u;

/* rows of 64 records a book of this capacity spans (the capacity class) */
inline int rows_for_cap(int cap) { return (cap + WAVE - 1) / WAVE; }


struct KArgs {
    /* configuration */
    int32_t n_envs, n_agents, max_cap, episode_len;
    uint64_t seed;
    int32_t exec_task, exec_q0, mm_q, dir_q;
    float pen, lam, rho;
    /* Avellaneda-Stoikov quote terms per risk-aversion choice g, tabled on the host in
     * device memory: [g] = gamma sigma^2, [9 + g] = (2 / gamma) ln(1 + gamma / kappa)
     * (a kernel-argument array indexed at run time would be copied to scratch) */
    const double *avst;
    int32_t kinds; /* 4 bits per agent */
    const int32_t *caps;
    /* messages */
    const int32_t *m_ts, *m_price, *m_qty, *m_oid, *m_tid, *m_tsec, *m_tns;
    const int64_t *m_off;
    int32_t m_steps;
    const int32_t *actions_in;
    /* outputs */
    int32_t *trades;
    const int64_t *trade_off;
    int64_t *trade_cursor;
    int32_t *n_trades;
    int64_t *fills;
    float *reward;
    float *obs;
    uint8_t *done;
    int32_t *actions_out;
    /* state */
    int32_t *bk[NF];
    int32_t *bk_n;
    int64_t *env_state, *agent_state, *counters, *stats;
    /* schedule */
    const int32_t *env_list;
    int32_t n_list;
    int32_t *work_ctr;
    int32_t t0, n_steps, capp, lds_words;
};

/* ------------------------------------------------------------------------------
 * A chunk of up to 64 messages staged in registers, message k in lane k: the dispatch
 * code (below), price, qty, oid, tid and the time reference of the message.  Fields of
 * message j are read into scalar registers where a handler needs them.
 * ---------------------------------------------------------------------------- */
/* dispatch code: side in bit 0, operation above it */
enum { OP_LIMIT = 0, OP_DELETE = 2, OP_PCANCEL = 4, OP_MARKET = 6, OP_EXECUTE = 8, OP_IGNORED = 10, OP_BAD = 12 };
/* Sec. 4 step 4 message semantics: a delete ignores its quantity and an ignored message
 * everything; a limit, market, partial cancel or execution needs a positive quantity;
 * other types are invalid */
__device__ __forceinline__ int op_code(int ts, int qty) {
    const int type = ts & 0xFF;
    int op = OP_BAD;
    if (type == T_LIMIT) op = OP_LIMIT;
    if (type == T_DELETE) op = OP_DELETE;
    if (type == T_PCANCEL) op = OP_PCANCEL;
    if (type == T_MARKET) op = OP_MARKET;
    if (type == T_EXECUTE) op = OP_EXECUTE;
    if (type == T_IGNORED) op = OP_IGNORED;
    if (qty <= 0 && type != T_DELETE && type != T_IGNORED) op = OP_BAD;
    return op | ((ts >> 8) & 1);
}
struct Staged {
    int c[6] = {0, 0, 0, 0, 0, 0};
    int j = 0;
    __device__ __forceinline__ int code() const { return rdlane(c[0], j); }
    __device__ __forceinline__ int price() const { return rdlane(c[1], j); }
    __device__ __forceinline__ int qty() const { return rdlane(c[2], j); }
    __device__ __forceinline__ int oid() const { return rdlane(c[3], j); }
    __device__ __forceinline__ int tid() const { return rdlane(c[4], j); }
    __device__ __forceinline__ int tref() const { return rdlane(c[5], j); }
};

/* ------------------------------------------------------------------------------
 * One environment run by one wavefront.
 * ---------------------------------------------------------------------------- */
struct Run {
    const KArgs &a;
    int32_t *L;  /* this wave's LDS (uniform) */
    int lane, cap, capp, e, A, t;
    /* book: live orders and best price per side */
    int n0, n1, best0, best1;
    /* per step, hot */
    int64_t mid_sum, st_buy, st_sell;
    int32_t mid_n, seq, st_last, last_tsec, last_tns;
    /* time references: of the last processed message (TREF_START before any in this
     * launch), the launch's start time it stands for, and the stream's first message */
    int32_t last_ref, start_tsec, start_tns;
    int64_t sbase;
    /* mid statistics run-length encoded: the messages since index mid_at all leave the
     * book with the same touch, contributing mid_c (best bid + best ask, or 0 when a side
     * is empty) and mid_f (1, or 0 when a side is empty) each */
    int64_t mid_c;
    int32_t mid_f, mid_at;
    /* trade records: this launch's part of the env's region starts at tr_base; records
     * produced so far in the launch, room left in the region, value at step start */
    int32_t *tr_base;
    int64_t tr_cur0;
    int32_t tr_next, tr_room, tr_step0;
    /* counters: lane k holds counter k */
    int64_t ctr;
    /* the agents' desired levels of the step, in registers: lane MAXLV i + k holds level k
     * of agent i (side, price, desired and resting quantity, the resting quantity the walk
     * has seen so far), lane i the level count of agent i */
    int lv_side, lv_price, lv_d, lv_r, lv_seen, lv_n;
    /* the agents' resting orders on side S at step start, best first: lane p holds the
     * p-th one as 8 x record index + owner's tid (the index kept current through the
     * cancel walk), and its price and quantity for the resting quantities measured before
     * the walk; al_n[S] counts them all, the first WAVE are held */
    int al_jt[2], al_px[2], al_q[2], al_n[2];

    __device__ Run(const KArgs &args, int32_t *lds, int env)
        : a(args), L(lds), lane(lane_id()), capp(uni(args.capp)), e(uni(env)), A(args.n_agents),
          n0(0), n1(0), best0(0), best1(0), mid_sum(0), mid_n(0), seq(0), last_ref(TREF_START), start_tsec(0),
          start_tns(0), sbase(0), mid_c(0), mid_f(0), mid_at(0) {
        cap = uni(a.caps[e]);
    }

    /* ---- LDS views.  Each side holds capp records of two int2 (price|qty, oid|tid),
     * both sides' records first, then both sides' time references (capp words each).
     * Record j counts from the worst order (j = 0) to the best (j = n - 1), so the top of
     * the book is at the end of the live range; record j of a row of 64 belongs to lane
     * j % 64. ---- */
    /* pair p of record i of side s (any index, e.g. uniform) */
    __device__ __forceinline__ int2 &U(int s, int p, int i) {
        return reinterpret_cast<int2 *>(L)[(s * capp + i) * REC + p];
    }
    /* time reference of record i of side s */
    __device__ __forceinline__ int32_t &T(int s, int i) { return L[2 * REC * 2 * capp + s * capp + i]; }
    __device__ __forceinline__ int32_t *X() { return L + 10 * capp; }
    __device__ __forceinline__ XL xl() const { return x_layout(A); }
    __device__ __forceinline__ int64_t *X64(int off) { return reinterpret_cast<int64_t *>(X() + off); }
    __device__ __forceinline__ int64_t *AG(int i) { return X64(xl().ag) + i * AGW; }
    __device__ __forceinline__ int64_t *FL(int i) { return X64(xl().fl) + i * 4; }
    __device__ __forceinline__ int64_t *ENV() { return X64(xl().env); }

    __device__ __forceinline__ int nsz(int s) const { return s ? n1 : n0; }
    __device__ __forceinline__ void count(int k, int64_t v) { ctr += (lane == k) ? v : 0; }

    /* ---- side-specialised views (S = 0 bids, 1 asks, known at compile time) ---- */
    template <int S> __device__ __forceinline__ int &nS() {
        if constexpr (S == 0) return n0; else return n1;
    }
    template <int S> __device__ __forceinline__ int &bestS() {
        if constexpr (S == 0) return best0; else return best1;
    }
    /* prices of side S compare as (price ^ km(S)): "equal or better" is "<=" for both */
    static constexpr int km(int s) { return s == 0 ? -1 : 0; }
    template <int S> __device__ __forceinline__ int2 &US(int p, int i) {
        int2 *base = reinterpret_cast<int2 *>(L) + (S == 0 ? 0 : capp * REC);
        return base[i * REC + p];
    }
    template <int S> __device__ __forceinline__ void refresh_bestS() {
        const int n = nS<S>();
        bestS<S>() = n > 0 ? uni(US<S>(0, n - 1).x) : 0;
        touch_changed();
    }
    /* the touch (best prices, or a side's emptiness) may have changed during message seq:
     * the messages of the closed run contribute the previous touch */
    __device__ __forceinline__ void mid_flush() {
        const int len = seq - mid_at;
        mid_sum += mid_c * len;
        mid_n += mid_f * len;
        mid_at = seq;
    }
    /* a uniform value kept in vector registers (its arithmetic then issues as VALU) */
    static __device__ __forceinline__ int64_t vreg64(int64_t x) {
        int lo = (int)x, hi = (int)(x >> 32);
        asm volatile("v_mov_b32 %0, %0" : "+v"(lo));
        asm volatile("v_mov_b32 %0, %0" : "+v"(hi));
        return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
    }
    static __device__ __forceinline__ int vreg32(int x) {
        asm volatile("v_mov_b32 %0, %0" : "+v"(x));
        return x;
    }
    __device__ __forceinline__ void touch_changed() {
        mid_flush();
        mid_f = min(n0, n1) > 0 ? 1 : 0;
        mid_c = vreg64(mid_f ? (int64_t)best0 + best1 : 0);
    }

    /* record i of side S (any index; the side's base is uniform) */
    template <int S> __device__ __forceinline__ int2 *RS(int i) {
        return reinterpret_cast<int2 *>(L) + (S * capp + i) * REC;
    }
    /* time reference of record i of side S */
    template <int S> __device__ __forceinline__ int32_t *TS(int i) { return L + 2 * REC * 2 * capp + S * capp + i; }
    /* record i of side S as one 128-bit value (price, qty, oid, tid) */
    template <int S> __device__ __forceinline__ int4 *RQ(int i) { return reinterpret_cast<int4 *>(L) + S * capp + i; }
    /* lanes whose price x is equal to or better than p on side S */
    template <int S> __device__ __forceinline__ uint64_t better_eq(int x, int p) {
        return S == 0 ? lanes_ge(x, p) : lanes_le(x, p);
    }

    /* ---- searches: rows from the top of the book down, stopping at the first hit.  Every
     * lane loads (indices clamped into the live range) and the lane range is a mask, so a
     * row costs one LDS load and no branches on the execution mask. ---- */
    /* highest record <= hi of side S whose field f (FO or FT) equals v, or -1; for oids
     * this is the first order with that id in priority order */
    template <int S> __device__ __forceinline__ int find_top(int f, int hi, int v) {
        const int32_t *col = reinterpret_cast<const int32_t *>(RS<S>(0)) + f;
        /* FIND_ROWS rows per LDS round trip (their loads are issued together): a cancel
         * whose order is gone (a quarter of the replayed messages) searches every row */
        for (int r = hi >> 6; r >= 0; r -= FIND_ROWS) {
            int x[FIND_ROWS];
#pragma unroll
            for (int k = 0; k < FIND_ROWS; ++k) {
                const int j = (max(r - k, 0) << 6) + lane;
                x[k] = col[min(j, hi) * (2 * REC)];
            }
#pragma unroll
            for (int k = 0; k < FIND_ROWS; ++k) {
                if (r - k < 0) return -1;
                const int j = ((r - k) << 6) + lane;
                const uint64_t m = lanes_eq(x[k], v) & lanes_le(j, hi);
                if (m) return ((r - k) << 6) + 63 - __builtin_clzll(m);
            }
        }
        return -1;
    }
    /* orders equal to or better than price p in the full rows r, r-1, ..., 0 of side S,
     * counted from the top while whole rows are */
    template <int S> __device__ __forceinline__ int count_rows(int r, int p) {
        int cnt = 0;
        for (; r >= 0; --r) {
            const int c = __popcll(better_eq<S>(RS<S>((r << 6) + lane)->x, p));
            cnt += c;
            if (c < WAVE) break;
        }
        return cnt;
    }
    /* orders of side S (n live) whose price is equal to or better than p: they are the
     * top records of the side */
    template <int S> __device__ __forceinline__ int count_ahead(int n, int p) {
        if (n == 0) return 0;
        const int rt = (n - 1) >> 6, top = n - (rt << 6);
        const int x = RS<S>(min((rt << 6) + lane, n - 1))->x;
        const int c = __popcll(better_eq<S>(x, p) & lanes_lt(lane, top));
        return c < top ? c : c + count_rows<S>(rt - 1, p);
    }

    /* ---- book edits: one pass over the rows they touch, loads of a row before its
     * stores; each lane moves one record ---- */
    /* rows r0 down to (ins >> 6): record j (ins < j, and j <= n in row r0) takes record j - 1 */
    template <int S> __device__ __forceinline__ void shift_up_rows(int r0, int ins) {
        for (int r = r0; r >= (ins >> 6); --r) {
            const int j = (r << 6) + lane;
            const int4 x = *RQ<S>(max(j - 1, 0));
            const int xt = *TS<S>(max(j - 1, 0));
            WAVE_SYNC();
            if (j > ins) {
                *RQ<S>(j) = x;
                *TS<S>(j) = xt;
            }
            WAVE_SYNC();
        }
    }
    /* one record written by lane 0 */
    template <int S> __device__ __forceinline__ void put(int i, int4 v, int vt) {
        if (lane == 0) {
            *RQ<S>(i) = v;
            *TS<S>(i) = vt;
        }
        WAVE_SYNC();
    }
    /* record k of side S (n live), below the top row rt = (n - 1) >> 6, leaves: [k+1, n)
     * moves down by one, row by row from k's row up; the top row from (o, ot), that row as
     * loaded before (lane l: record 64 rt + l) */
    template <int S> __device__ __forceinline__ void remove_below_top(int k, int n, int4 o, int ot) {
        const int rt = (n - 1) >> 6;
        for (int r = k >> 6; r < rt; ++r) {
            const int j = (r << 6) + lane;
            const int4 x = *RQ<S>(j + 1);
            const int xt = *TS<S>(j + 1);
            WAVE_SYNC();
            if (j >= k) {
                *RQ<S>(j) = x;
                *TS<S>(j) = xt;
            }
            WAVE_SYNC();
        }
        const int j = (rt << 6) + lane;
        const int4 u = make_int4(shl1(o.x), shl1(o.y), shl1(o.z), shl1(o.w));
        const int ut = shl1(ot);
        if (j < n - 1) {
            *RQ<S>(j) = u;
            *TS<S>(j) = ut;
        }
        WAVE_SYNC();
    }
    /* full side (n = cap): the worst order (record 0) leaves, [1, ins) moves down by one and
     * the new order takes record ins - 1 (ins >= 1) */
    template <int S> __device__ __forceinline__ void evict_insert(int ins, int4 v, int vt) {
        for (int r = 0; r <= (ins - 1) >> 6; ++r) {
            const int j = (r << 6) + lane;
            const int4 x = *RQ<S>(min(j + 1, ins - 1));
            const int xt = *TS<S>(min(j + 1, ins - 1));
            WAVE_SYNC();
            if (j < ins - 1) {
                *RQ<S>(j) = x;
                *TS<S>(j) = xt;
            }
            WAVE_SYNC();
        }
        put<S>(ins - 1, v, vt);
    }

    /* ---- fills (uniform accumulation in LDS by lane 0) ---- */
    __device__ __forceinline__ void add_fill(int tid, int buy, int64_t q, int64_t notional) {
        if ((unsigned)(tid - 1) < (unsigned)A) { /* agent tids are 1..A */
            if (lane == 0) {
                int64_t *f = FL(tid - 1) + (buy ? 0 : 2);
                f[0] += q;
                f[1] += notional;
            }
            WAVE_SYNC();
        }
    }

    /* ---- trade records (written by lane 0) ---- */
    __device__ __forceinline__ void write_trade(int k, int price, int q, int agg_oid, int pas_oid,
                                                int agg_tid, int pas_tid, int side) {
        const int rec = tr_next + k;
        if (rec < tr_room) {
            if (lane == 0) {
                int4 *p = reinterpret_cast<int4 *>(tr_base + (int64_t)rec * LOB_TRADE_WORDS);
                p[0] = make_int4(price, q, agg_oid, pas_oid);
                p[1] = make_int4(agg_tid, pas_tid, side | (seq << 1), t);
            }
        }
    }

    /* ---- matching: an incoming order of side S against the opposite side while it
     * crosses (market orders cross at any price); trades at the resting price, best
     * first.  The best order is read first (one broadcast read); when it alone does not
     * fill the order, the 64 best orders are loaded at once, lane l holding the l-th
     * best, an inclusive prefix sum of the crossing quantities over the lanes finds
     * where the order is filled, and the lanes up to that one write their trade records
     * together (a sweep beyond 64 orders takes the next 64).  Returns the unmatched
     * remainder. ---- */
    template <int S, bool MARKET>
    __device__ __forceinline__ int match(int p, int q, int agg_oid, int agg_tid) {
        constexpr int O = 1 - S;
        const int n_opp = nS<O>();
        if (n_opp == 0) return q;
        const int kp = p ^ km(O);
        if (!MARKET && (bestS<O>() ^ km(O)) > kp) return q;
        int no = n_opp, rem = q, ntr = 0, last_price = 0;
        /* the notional of the fills is needed only for an agent's own fill (replayed
         * orders have no agent tid) */
        const bool agg_agent = (unsigned)(agg_tid - 1) < (unsigned)A;
        int64_t notional = 0;
        /* lane 0: the best order, the other lanes the second best (clamped) */
        const int4 bo = *RQ<O>(max(no - 1 - min(lane, 1), 0));
        /* prices of the last rows read, lane l the order no_row - 1 - l: the new best
         * order after the fills is among them unless a whole row was consumed */
        int rx = bo.x, no_row = no;
        const int bq = rdlane(bo.y, 0);
        if (bq >= rem) {
            /* it fills the order (the common case): one trade, no row load */
            const int bp = rdlane(bo.x, 0), bt = rdlane(bo.w, 0);
            write_trade(0, bp, rem, agg_oid, rdlane(bo.z, 0), agg_tid, bt, S);
            add_fill(bt, S != 0, rem, (int64_t)rem * bp);
            if (rem < bq) {
                if (lane == 0) RQ<O>(no - 1)->y = bq - rem;
                WAVE_SYNC();
            } else {
                no -= 1;
            }
            notional = (int64_t)rem * bp;
            last_price = bp;
            ntr = 1;
            rem = 0;
        } else for (;;) {
            /* lane l: the l-th best order of the opposite side (record no - 1 - l) */
            const int j = no - 1 - lane;
            const int4 r = *RQ<O>(max(j, 0));
            rx = r.x;
            no_row = no;
            const bool cross = j >= 0 && (MARKET || (r.x ^ km(O)) <= kp);
            const uint64_t ncm = ballot(!cross);
            if (ncm & 1) break; /* after a row of fills: the new best order does not cross */
            int kd, kn, nt;
            unsigned inc = 0, exc = 0;
            if (rdlane(r.y, 0) >= rem) {
                kd = 0; /* the row's best order fills the rest */
                kn = nt = 1;
            } else {
                inc = scan_sat(cross ? (unsigned)r.y : 0u);
                exc = (unsigned)shr1((int)inc);
                const uint64_t dm = ballot(cross && inc >= (unsigned)rem);
                kn = ncm ? (int)__builtin_ctzll(ncm) : WAVE; /* first order that does not cross */
                kd = dm ? (int)__builtin_ctzll(dm) : WAVE;   /* the order that fills the rest */
                nt = min(kd + 1, kn);                       /* orders traded against */
            }
            const int x = lane == kd ? rem - (int)exc : r.y; /* lane l < nt trades x */
            const int rec = tr_next + ntr + lane;
            if (lane < nt && rec < tr_room) {
                int4 *pt = reinterpret_cast<int4 *>(tr_base + (int64_t)rec * LOB_TRADE_WORDS);
                pt[0] = make_int4(r.x, x, agg_oid, r.z);
                pt[1] = make_int4(agg_tid, r.w, S | (seq << 1), t);
            }
            /* passive fills of agents' orders among them (rare) */
            uint64_t am = ballot(lane < nt && (unsigned)(r.w - 1) < (unsigned)A);
            while (am) {
                const int l = (int)__builtin_ctzll(am);
                am &= am - 1;
                const int px = rdlane(x, l);
                add_fill(rdlane(r.w, l), S != 0, px, (int64_t)px * rdlane(r.x, l));
            }
            if (agg_agent)
                for (int l = 0; l < nt; ++l) notional += (int64_t)rdlane(x, l) * rdlane(r.x, l);
            last_price = rdlane(r.x, nt - 1);
            ntr += nt;
            if (kd < kn) {
                /* filled at lane kd: that order keeps the rest of its quantity, if any */
                const int qk = rdlane(r.y, kd), xk = rdlane(x, kd);
                if (xk < qk) {
                    if (lane == kd) RQ<O>(j)->y = qk - xk;
                    WAVE_SYNC();
                    no -= kd;
                } else {
                    no -= kd + 1;
                }
                rem = 0;
                break;
            }
            no -= nt;
            rem -= rdlane((int)inc, nt - 1);
            if (kn < WAVE || no == 0) break;
        }
        if (agg_agent) add_fill(agg_tid, S == 0, q - rem, notional);
        if (no != n_opp) {
            nS<O>() = no;
            const int l = no_row - no; /* lane of the new best order in rx */
            if (no > 0 && l < WAVE) {
                bestS<O>() = rdlane(rx, l);
                touch_changed();
            } else {
                refresh_bestS<O>();
            }
        }
        tr_next += ntr;
        if (S == 0) st_buy += q - rem; else st_sell += q - rem;
        st_last = last_price;
        return rem;
    }

    /* ---- rest a limit remainder on its own side S (after all orders at an equal or
     * better price); a full side evicts its worst order if the price is strictly
     * better than that order's, else the remainder is dropped. ---- */
    template <int S>
    __device__ __forceinline__ void rest(int p, int q, int oid, int tid, const Staged &m) {
        const int n = nS<S>();
        int cnt;
        if (n < cap) {
            if (n > 0) {
                /* the top row of the insertion, rt = n >> 6, loaded once: lane l holds
                 * record j - 1 for j = 64 rt + l (clamped into the live range).  Lanes 1..top
                 * hold the row's live records, so they also give the count from the top. */
                const int rt = n >> 6, top = n - (rt << 6);
                const int j = (rt << 6) + lane;
                const int js = min(max(j - 1, 0), n - 1);
                const int4 y = *RQ<S>(js);
                const int yt = *TS<S>(js);
                cnt = __popcll(better_eq<S>(y.x, p) & ~1ull & lanes_le(lane, top)); /* lanes 1..top */
                if (cnt == top) cnt += count_rows<S>(rt - 1, p);
                const int ins = n - cnt;
                WAVE_SYNC();
                if ((ins >> 6) == rt) {
                    /* the edit stays in row rt: lanes above ins take the record below,
                     * lane ins the new order, in one store */
                    const int tr = m.tref();
                    const bool me = j == ins;
                    const int4 v = make_int4(me ? p : y.x, me ? q : y.y, me ? oid : y.z, me ? tid : y.w);
                    const int vt = me ? tr : yt;
                    if ((unsigned)(j - ins) <= (unsigned)(n - ins)) {
                        *RQ<S>(j) = v;
                        *TS<S>(j) = vt;
                    }
                    WAVE_SYNC();
                } else {
                    if ((unsigned)(j - ins - 1) < (unsigned)(n - ins)) {
                        *RQ<S>(j) = y;
                        *TS<S>(j) = yt;
                    }
                    WAVE_SYNC();
                    shift_up_rows<S>(rt - 1, ins);
                    put<S>(ins, make_int4(p, q, oid, tid), m.tref());
                }
            } else {
                cnt = 0;
                put<S>(0, make_int4(p, q, oid, tid), m.tref());
            }
            nS<S>() = n + 1;
        } else if (n <= WAVE) {
            /* a full side of one row, loaded once (lane l: record l): the worst order is
             * lane 0, the orders ahead of the new one are counted from the same load, and
             * on an eviction lanes below ins - 1 take the record above them, lane ins - 1
             * the new order, in one store */
            const int4 y = *RQ<S>(min(lane, n - 1));
            const int yt = *TS<S>(min(lane, n - 1));
            const int wp = rdlane(y.x, 0);
            if ((p ^ km(S)) >= (wp ^ km(S))) {
                count(C_DROP, 1);
                count(C_DROPPED_QTY, q);
                return;
            }
            count(C_EVICT, 1);
            count(C_EVICTED_QTY, rdlane(y.y, 0));
            cnt = __popcll(better_eq<S>(y.x, p) & lanes_lt(lane, n));
            const int ins = n - cnt;
            const int tr = m.tref();
            const bool me = lane == ins - 1;
            const int4 u = make_int4(shl1(y.x), shl1(y.y), shl1(y.z), shl1(y.w));
            const int ut = shl1(yt);
            const int4 v = make_int4(me ? p : u.x, me ? q : u.y, me ? oid : u.z, me ? tid : u.w);
            const int vt = me ? tr : ut;
            WAVE_SYNC();
            if (lane < ins) {
                *RQ<S>(lane) = v;
                *TS<S>(lane) = vt;
            }
            WAVE_SYNC();
        } else {
            const int2 w = *RS<S>(0);
            const int wp = uni(w.x);
            if ((p ^ km(S)) >= (wp ^ km(S))) {
                count(C_DROP, 1);
                count(C_DROPPED_QTY, q);
                return;
            }
            count(C_EVICT, 1);
            count(C_EVICTED_QTY, uni(w.y));
            cnt = count_ahead<S>(n, p);
            evict_insert<S>(n - cnt, make_int4(p, q, oid, tid), m.tref());
        }
        if (cnt == 0) {
            bestS<S>() = p;
            touch_changed();
        }
    }

    /* ---- messages naming a resting order: the first order with this id (priority order)
     * on side S.  A delete removes it; a partial cancel takes up to qty from it; a
     * replayed execution trades up to qty of it at its price against an anonymous
     * aggressor of the other side.  The top row is loaded whole; a hit there is removed
     * from registers (each lane takes the record of the lane above it), deeper hits search
     * and shift row by row. ---- */
    enum { CX_DELETE = 0, CX_PARTIAL = 1, CX_EXECUTE = 2 };
    /* the execution of x of the order (price, tid, id oid) of side S */
    template <int S> __device__ __forceinline__ void executed(int price, int tid, int oid, int x) {
        write_trade(0, price, x, 0, oid, 0, tid, 1 - S);
        tr_next += 1;
        add_fill(tid, S == 0, x, (int64_t)x * price);
        if (S == 1) st_buy += x; else st_sell += x;
        st_last = price;
    }
    /* returns the index the removed order had, or -1 (no order left the book) */
    template <int S, int MODE>
    __device__ __forceinline__ int cancel(int qty, int oid) {
        const int n = nS<S>();
        if (n == 0) {
            count(C_MISS, 1);
            return -1;
        }
        const int rt = (n - 1) >> 6;
        const int j = (rt << 6) + lane;
        int4 o = *RQ<S>(min(j, n - 1));
        int ot = *TS<S>(min(j, n - 1));
        /* the whole top row (records and time references) arrives in the one LDS round
         * trip that the id comparison waits for anyway; a hit then moves it from
         * registers */
        asm volatile("" : "+v"(o.x), "+v"(o.y), "+v"(o.z), "+v"(o.w), "+v"(ot));
        const uint64_t mt = lanes_eq(o.z, oid) & lanes_lt(j, n);
        int k;
        if (mt) {
            k = (rt << 6) + 63 - __builtin_clzll(mt);
            if (MODE != CX_DELETE) {
                const int cq = rdlane(o.y, k & 63);
                const int x = min(qty, cq);
                if (MODE == CX_EXECUTE) executed<S>(rdlane(o.x, k & 63), rdlane(o.w, k & 63), oid, x);
                const int left = cq - x;
                if (left > 0) {
                    if (lane == 0) RS<S>(k)->y = left;
                    WAVE_SYNC();
                    return -1;
                }
            }
            const int4 u = make_int4(shl1(o.x), shl1(o.y), shl1(o.z), shl1(o.w));
            const int ut = shl1(ot);
            WAVE_SYNC();
            if ((unsigned)(j - k) < (unsigned)(n - 1 - k)) {
                *RQ<S>(j) = u;
                *TS<S>(j) = ut;
            }
            WAVE_SYNC();
            nS<S>() = n - 1;
            if (k == n - 1) {
                /* the best order left: the next best is the record below it, in the
                 * loaded row unless k opened the row */
                if (k & 63) {
                    bestS<S>() = rdlane(o.x, (k & 63) - 1);
                    touch_changed();
                } else {
                    refresh_bestS<S>();
                }
            }
            return k;
        } else {
            k = find_top<S>(FO, (rt << 6) - 1, oid);
            if (k < 0) {
                count(C_MISS, 1);
                return -1;
            }
            if (MODE != CX_DELETE) {
                const int4 rk = *RQ<S>(k);
                const int cq = uni(rk.y);
                const int x = min(qty, cq);
                if (MODE == CX_EXECUTE) executed<S>(uni(rk.x), uni(rk.w), oid, x);
                const int left = cq - x;
                if (left > 0) {
                    if (lane == 0) RS<S>(k)->y = left;
                    WAVE_SYNC();
                    return -1;
                }
            }
            remove_below_top<S>(k, n, o, ot);
        }
        /* below the top row: the best order stays */
        nS<S>() = n - 1;
        return k;
    }

    /* ---- one message of the step sequence: m.code says which handler (the operation
     * and side, with invalid messages already folded into OP_BAD); each test is a single
     * comparison of that uniform code ---- */
    template <int S> __device__ __forceinline__ void limit(const Staged &m) {
        const int price = m.price(), qty = m.qty(), oid = m.oid(), tid = m.tid();
        const int q = match<S, false>(price, qty, oid, tid);
        if (q > 0) rest<S>(price, q, oid, tid, m);
    }
    template <int S> __device__ __forceinline__ void market(const Staged &m) {
        const int q = match<S, true>(0, m.qty(), m.oid(), m.tid());
        if (q > 0) count(C_MARKET_UNFILLED, q);
    }
    __device__ __forceinline__ void process(const Staged &m) {
        const int code = m.code();
        if (code < OP_DELETE) {
            if (code == OP_LIMIT) limit<0>(m);
            else limit<1>(m);
        } else if (code < OP_MARKET) {
            if (code < OP_PCANCEL) {
                if (code == OP_DELETE) cancel<0, CX_DELETE>(0, m.oid());
                else cancel<1, CX_DELETE>(0, m.oid());
            } else {
                if (code == OP_PCANCEL) cancel<0, CX_PARTIAL>(m.qty(), m.oid());
                else cancel<1, CX_PARTIAL>(m.qty(), m.oid());
            }
        } else if (code < OP_EXECUTE) {
            if (code == OP_MARKET) market<0>(m);
            else market<1>(m);
        } else if (code < OP_IGNORED) {
            if (code == OP_EXECUTE) cancel<0, CX_EXECUTE>(m.qty(), m.oid());
            else cancel<1, CX_EXECUTE>(m.qty(), m.oid());
        } else if (code < OP_BAD) {
            count(C_IGNORED, 1);
        } else {
            count(C_BAD, 1);
        }
        after_message();
    }
    /* per message of the sequence: the message index (the mid statistics follow the
     * touch, see touch_changed) */
    __device__ __forceinline__ void after_message() { seq += 1; }

    /* ---- desired levels of agent ai (registers, lane MAXLV ai + k: level k) ---- */
    /* the lane of agent ai's level (side, price) among its first nlv, or -1 */
    __device__ __forceinline__ int find_level(int ai, int nlv, int side, int price) {
        const uint64_t m = ballot((unsigned)(lane - MAXLV * ai) < (unsigned)nlv && lv_side == side && lv_price == price);
        return m ? (int)__builtin_ctzll(m) : -1;
    }
    __device__ __forceinline__ void add_level(int ai, int &nlv, int side, int price, int qty) {
        const int l = find_level(ai, nlv, side, price);
        if (l >= 0) {
            lv_d += lane == l ? qty : 0;
        } else if (nlv < MAXLV) {
            if (lane == MAXLV * ai + nlv) {
                lv_side = side; lv_price = price; lv_d = qty; lv_r = 0; lv_seen = 0;
            }
            nlv += 1;
        }
    }

    /* every agent's resting orders on side S, best first, into the al_* registers: two
     * rows of whole records per LDS round trip, a ballot of the agents' tids per row */
    template <int S> __device__ __forceinline__ void agent_scan() {
        const int n = nS<S>();
        int c = 0, ajt = -1, apx = 0, aq = 0;
        auto take = [&](int r, const int4 &x) {
            uint64_t m = ballot((r << 6) + lane < n && (unsigned)(x.w - 1) < (unsigned)A);
            while (m) {
                const int l = 63 - __builtin_clzll(m);
                m &= ~(1ull << l);
                if (c < WAVE) {
                    const bool me = lane == c;
                    const int px = rdlane(x.x, l), q = rdlane(x.y, l), tid = rdlane(x.w, l);
                    ajt = me ? 8 * ((r << 6) + l) + tid : ajt;
                    apx = me ? px : apx;
                    aq = me ? q : aq;
                }
                c += 1;
            }
        };
        for (int r = (n - 1) >> 6; r >= 0; r -= 2) {
            const int4 x0 = *RQ<S>(min((r << 6) + lane, n - 1));
            const int4 x1 = *RQ<S>(max(((r - 1) << 6) + lane, 0));
            take(r, x0);
            if (r >= 1) take(r - 1, x1);
        }
        al_jt[S] = ajt; al_px[S] = apx; al_q[S] = aq; al_n[S] = c;
    }

    /* the agent's resting quantity at each of its desired levels on side S: its orders
     * among the held ones, then (more than WAVE agent orders on the side) a search below
     * the last held one */
    template <int S> __device__ __forceinline__ void resting_side(int i, int nlv, int tid) {
        uint64_t m = ballot(lane < min(al_n[S], WAVE) && (al_jt[S] & 7) == tid);
        while (m) {
            const int p = (int)__builtin_ctzll(m);
            m &= m - 1;
            const int l = find_level(i, nlv, S, rdlane(al_px[S], p));
            if (l >= 0) lv_r += lane == l ? rdlane(al_q[S], p) : 0;
        }
        if (al_n[S] > WAVE) {
            int hi = (rdlane(al_jt[S], WAVE - 1) >> 3) - 1;
            for (;;) {
                const int j = find_top<S>(FT, hi, tid);
                if (j < 0) break;
                const int2 pq = US<S>(0, j);
                const int l = find_level(i, nlv, S, uni(pq.x));
                if (l >= 0) lv_r += lane == l ? uni(pq.y) : 0;
                hi = j - 1;
            }
        }
    }

    /* Sec. 4 step 1, from the book at step start, for agent i: decode its action into
     * desired levels (Sec. 4.1), measure its resting quantity at each of them and append
     * its new orders (the difference to the desired quantity, then any market order) to
     * the action block.  The cancels are emitted later, in the message loop. */
    __device__ __forceinline__ void agent_start(int i, int act, int bb0, int ba0, int &nact) {
        const int kind = (a.kinds >> (4 * i)) & 15;
        const int tid = i + 1;
        int nlv = 0;
        int64_t mkt = 0;
        if (kind == LOB_AGENT_EXEC) {
            /* sell task: prices far touch, mid (rounded up), near touch, near+2; 1x/2x/5x
             * the order quantity; a 4-level ladder; clipped in order to the remainder */
            int64_t left = uni64(AG(i)[2]);
            const int64_t q0 = a.exec_q0;
            const int64_t m2 = (int64_t)bb0 + ba0;
            const int mid_up = (int)(m2 >= 0 ? (m2 + 1) / 2 : -((-m2) / 2));
            int np = 0;
            int pp[4] = {0, 0, 0, 0};
            int64_t pq[4] = {0, 0, 0, 0};
            bool market = false;
            switch (act) {
            case 1: market = true; np = 1; pq[0] = q0; break;
            case 2: np = 1; pp[0] = bb0; pq[0] = q0; break;
            case 3: np = 1; pp[0] = mid_up; pq[0] = q0; break;
            case 4: np = 1; pp[0] = ba0; pq[0] = q0; break;
            case 5: np = 1; pp[0] = ba0 + 2; pq[0] = q0; break;
            case 6: np = 1; pp[0] = ba0; pq[0] = 2 * q0; break;
            case 7: np = 1; pp[0] = ba0; pq[0] = 5 * q0; break;
            case 8:
                np = 4;
                pp[0] = ba0; pp[1] = ba0 + 1; pp[2] = ba0 + 2; pp[3] = ba0 + 3;
                pq[0] = pq[1] = pq[2] = pq[3] = q0;
                break;
            default: break;
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (k < np) {
                    const int64_t q = min(pq[k], left);
                    left -= q;
                    if (q > 0) {
                        if (market) mkt += q;
                        else add_level(i, nlv, 1, pp[k], (int)q);
                    }
                }
            }
        } else if (kind == LOB_AGENT_MM_SPREADSKEW) {
            /* spread-skew table: always two-sided, spread 1/3/5 ticks around the mid,
             * skew -1/0/+1; never crossing the step-start touch */
            const int spread = act < 3 ? 1 : (act < 6 ? 3 : 5);
            const int skew = act - 3 * (act / 3) - 1;
            const int64_t m2 = (int64_t)bb0 + ba0;
            const int64_t bid = floor_div2(m2 - spread) + skew;
            const int64_t ask = -floor_div2(-(m2 + spread)) + skew;
            add_level(i, nlv, 0, (int)min(bid, (int64_t)ba0 - 1), a.mm_q);
            add_level(i, nlv, 1, (int)max(ask, (int64_t)bb0 + 1), a.mm_q);
        } else if (kind == LOB_AGENT_MM_AVST || kind == LOB_AGENT_MM_AS) {
            /* Avellaneda-Stoikov: reservation price mid - q gamma sigma^2 (T - t) and spread
             * gamma sigma^2 (T - t) + (2 / gamma) ln(1 + gamma / kappa), q the inventory in
             * quote lots; the baseline takes gamma0 (choice 4) */
            const int g = kind == LOB_AGENT_MM_AS ? 4 : act;
            const double q = (double)uni64(AG(i)[0]) / (double)a.mm_q;
            const double tau = (double)(a.episode_len - t);
            const double mid = (double)((int64_t)bb0 + ba0) * 0.5;
            const double avA = a.avst[g], avB = a.avst[9 + g];
            const double r = mid - q * avA * tau;
            const double d = avA * tau + avB;
            const int bid = quote_price(floor(r - d * 0.5));
            const int ask = quote_price(ceil(r + d * 0.5));
            add_level(i, nlv, 0, (int)min((int64_t)bid, (int64_t)ba0 - 1), a.mm_q);
            add_level(i, nlv, 1, (int)max((int64_t)ask, (int64_t)bb0 + 1), a.mm_q);
        } else if (kind == LOB_AGENT_EXEC_TWAP) {
            /* TWAP: the shortfall to ceil(task (t + 1) / T) executed, at the best bid */
            const int64_t task = a.exec_task, rem = uni64(AG(i)[2]);
            const int64_t target = (task * (int64_t)(t + 1) + a.episode_len - 1) / a.episode_len;
            const int64_t q = min(max(target - (task - rem), (int64_t)0), rem);
            if (q > 0) add_level(i, nlv, 1, bb0, (int)q);
        } else if (kind == LOB_AGENT_MM || kind == LOB_AGENT_MM_BUYSELL) {
            /* fixed-quantity quotes: bid = bb - ob (below the best ask), ask = ba + oa
             * (above the best bid); action 8 ladders offsets 0..3 on both sides */
            const int q = a.mm_q;
            int ob = 0, oa = 0;
            bool hb = false, ha = false;
            switch (act) {
            case 1: hb = ha = true; ob = 2; oa = 2; break;
            case 2: hb = ha = true; ob = 4; oa = 4; break;
            case 3: hb = ha = true; ob = -1; oa = -1; break;
            case 4: hb = true; ob = 2; break;
            case 5: ha = true; oa = 2; break;
            case 6: hb = ha = true; ob = 5; oa = -1; break;
            case 7: hb = ha = true; ob = -1; oa = 5; break;
            default: break;
            }
            if (act == 8) {
                for (int o = 0; o < 4; ++o) add_level(i, nlv, 0, min(bb0 - o, ba0 - 1), q);
                for (int o = 0; o < 4; ++o) add_level(i, nlv, 1, max(ba0 + o, bb0 + 1), q);
            } else {
                if (hb) add_level(i, nlv, 0, min(bb0 - ob, ba0 - 1), q);
                if (ha) add_level(i, nlv, 1, max(ba0 + oa, bb0 + 1), q);
            }
        } else {
            /* directional: take the opposite touch with a fixed quantity */
            if (act == 1) add_level(i, nlv, 0, ba0, a.dir_q);
            if (act == 2) add_level(i, nlv, 1, bb0, a.dir_q);
        }
        if (lane == i) lv_n = nlv;

        /* resting quantity of this agent at each desired level (step start) */
        if (nlv > 0) {
            resting_side<0>(i, nlv, tid);
            resting_side<1>(i, nlv, tid);
        }
        /* new orders; order ids from the agent's counter */
        int64_t *g = AG(i);
        for (int k = 0; k <= nlv; ++k) {
            int type, side, price, qty;
            if (k < nlv) {
                const int l = MAXLV * i + k;
                const int D = rdlane(lv_d, l), R = rdlane(lv_r, l);
                if (D <= R) continue;
                type = T_LIMIT; side = rdlane(lv_side, l); price = rdlane(lv_price, l); qty = D - R;
            } else {
                if (mkt <= 0) continue;
                type = T_MARKET; side = 1; price = 0; qty = (int)mkt;
            }
            const int64_t c = uni64(g[3]);
            const int oid = (int)((1u << 30) | ((uint32_t)i << 26) | (uint32_t)(c & ((1 << 26) - 1)));
            if (lane == 0) {
                int32_t *m = X() + xl().act + nact * 8;
                m[0] = type | (side << 8); m[1] = price; m[2] = qty; m[3] = oid;
                m[4] = tid; m[5] = last_ref; m[6] = 0;
                g[3] = c + 1;
            }
            WAVE_SYNC();
            nact += 1;
        }
    }

    /* ---- observation features from the book (LDS accumulators) ---- */
    __device__ __forceinline__ void book_obs(int bb, int ba) {
        int64_t *O = X64(xl().obk);
        if (lane < 22 + 3 * A) O[lane] = 0;
        WAVE_SYNC();
        for (int s = 0; s < 2; ++s) {
            const int n = nsz(s);
            int64_t tot = 0;
            for (int r = 0; (r << 6) < n; ++r) {
                const int i = (r << 6) + lane;
                if (i < n) {
                    const int2 pq = U(s, 0, i);
                    const int td = U(s, 1, i).y;
                    const int64_t d = s == 0 ? (int64_t)bb - pq.x : (int64_t)pq.x - ba;
                    if (d >= 0 && d <= 9)
                        atomicAdd(reinterpret_cast<unsigned long long *>(O + s * 10 + d), (unsigned long long)pq.y);
                    if (td >= 1 && td <= A) {
                        atomicAdd(reinterpret_cast<unsigned long long *>(O + 22 + 3 * (td - 1) + s),
                                  (unsigned long long)pq.y);
                        atomicAdd(reinterpret_cast<unsigned long long *>(O + 22 + 3 * (td - 1) + 2), 1ull);
                    }
                    tot += pq.y;
                }
            }
            tot = wave_sum64(tot);
            WAVE_SYNC();
            if (lane == 0) O[20 + s] = tot;
            WAVE_SYNC();
        }
    }
    /* the 40 features of every agent from the state in LDS, written to base [A][n_envs][40] */
    __device__ __forceinline__ void write_obs(float *base) {
        const int64_t *E = ENV();
        const int64_t *S = X64(xl().st);
        const int bb = (int)uni64(E[0]), ba = (int)uni64(E[1]);
        book_obs(bb, ba);
        const int64_t *O = X64(xl().obk);
        const int64_t mid2 = (int64_t)bb + ba;
        const int64_t strades = uni64(S[2]);
        /* lane f forms feature f: every value it may need is loaded first (uniform values
         * and one per-lane read of the book features), then the lane selects its own, so
         * that no lane waits on a load another lane's feature needs */
        const int f = lane;
        const int64_t e3 = uni64(E[3]), e6 = uni64(E[6]), e7 = uni64(E[7]);
        const int64_t s0 = uni64(S[0]), s1 = uni64(S[1]), s3 = uni64(S[3]);
        const int64_t ob = O[(f >= 3 && f <= 24) ? f - 3 : 0];
        int64_t vc = 0; /* the features that do not depend on the agent */
        vc = f == 0 ? (int64_t)ba - bb : vc;
        vc = f == 1 ? e7 : vc;
        vc = f == 2 ? mid2 - e3 : vc;
        vc = (f >= 3 && f <= 24) ? ob : vc;
        vc = f == 25 ? (int64_t)n0 : vc;
        vc = f == 26 ? (int64_t)n1 : vc;
        vc = f == 27 ? s0 : vc;
        vc = f == 28 ? s1 : vc;
        vc = f == 29 ? strades : vc;
        vc = f == 30 ? (strades > 0 ? 2 * s3 - mid2 : 0) : vc;
        vc = f == 34 ? (int64_t)a.episode_len - e6 : vc;
        for (int i = 0; i < A; ++i) {
            const int kind = (a.kinds >> (4 * i)) & 15;
            const int64_t *g = AG(i);
            const int64_t g0 = uni64(g[0]), g1 = uni64(g[1]), g2 = uni64(g[2]), g4 = uni64(g[4]), g5 = uni64(g[5]);
            const int64_t oa = O[22 + 3 * i + min(max(f - 35, 0), 2)];
            int64_t v = vc;
            v = (f >= 35 && f <= 37) ? oa : v;
            v = f == 31 ? g0 : v;
            v = f == 32 ? g1 : v;
            v = f == 33 ? (exec_kind(kind) ? g2 : 0) : v;
            v = f == 38 ? g4 : v;
            v = f == 39 ? g5 : v;
            if (f < LOB_OBS_DIM) base[((int64_t)i * a.n_envs + e) * LOB_OBS_DIM + f] = (float)v;
        }
    }

    /* ---- load / store of the env (books in HBM are in priority order, best first) ---- */
    __device__ __forceinline__ void load() {
        const int64_t gb = (int64_t)e * 2;
        n0 = min(uni(a.bk_n[gb]), cap);
        n1 = min(uni(a.bk_n[gb + 1]), cap);
        for (int s = 0; s < 2; ++s) {
            const int n = nsz(s);
            const int64_t off = (gb + s) * a.max_cap;
            for (int i = lane; i < n; i += WAVE) {
                const int j = n - 1 - i;
                U(s, 0, j) = make_int2(a.bk[FP][off + i], a.bk[FQ][off + i]);
                U(s, 1, j) = make_int2(a.bk[FO][off + i], a.bk[FT][off + i]);
                T(s, j) = TREF_LOADED | i; /* its time stays in the books in memory */
            }
        }
        /* env state, statistics and agent state into LDS, counters into lanes */
        if (lane < ENVW) ENV()[lane] = a.env_state[(int64_t)e * ENVW + lane];
        if (lane < STW) X64(xl().st)[lane] = a.stats[(int64_t)e * STW + lane];
        if (lane < A * AGW) AG(0)[lane] = a.agent_state[(int64_t)e * A * AGW + lane];
        ctr = lane < NCTR ? a.counters[(int64_t)e * LOB_N_COUNTERS + lane] : 0;
        WAVE_SYNC();
        refresh_bestS<0>();
        refresh_bestS<1>();
        t = (int32_t)uni64(ENV()[6]);
        last_tsec = (int32_t)uni64(ENV()[4]);
        last_tns = (int32_t)uni64(ENV()[5]);
        last_ref = TREF_START;
        start_tsec = last_tsec;
        start_tns = last_tns;
        sbase = a.m_off ? uni64(a.m_off[(int64_t)e * (a.m_steps + 1)]) : 0;
        tr_cur0 = a.trade_cursor ? uni64(a.trade_cursor[e]) : 0;
        tr_next = 0;
        tr_base = nullptr;
        tr_room = 0;
        if (a.trades) {
            const int64_t b0 = a.trade_off[e] + tr_cur0;
            const int64_t room = a.trade_off[e + 1] - b0;
            tr_room = (int)max(min(room, (int64_t)1 << 30), -((int64_t)1 << 30));
            if (room > 0) tr_base = a.trades + b0 * LOB_TRADE_WORDS;
        }
    }
    __device__ __forceinline__ void store() {
        WAVE_SYNC();
        const int64_t gb = (int64_t)e * 2;
        constexpr int MAXR = LOB_MAX_CAP / WAVE;
        for (int s = 0; s < 2; ++s) {
            const int n = nsz(s);
            const int64_t off = (gb + s) * a.max_cap;
            /* the orders' times, from their references, into registers: every read of the
             * side's old time slots comes before any write to them */
            int ts[MAXR], tn[MAXR];
#pragma unroll
            for (int r = 0; r < MAXR; ++r) {
                const int i = (r << 6) + lane;
                ts[r] = 0;
                tn[r] = 0;
                if (i < n) {
                    const int tr = T(s, n - 1 - i);
                    if (tr >= 0) {
                        const int64_t g = sbase + tr;
                        ts[r] = a.m_tsec[g];
                        tn[r] = a.m_tns[g];
                    } else if (tr == TREF_START) {
                        ts[r] = start_tsec;
                        tn[r] = start_tns;
                    } else {
                        const int64_t k = off + (tr & 0x3FFFFFFF);
                        ts[r] = a.bk[FS][k];
                        tn[r] = a.bk[FN][k];
                    }
                }
            }
            __builtin_amdgcn_s_waitcnt(0x0F70); /* vmcnt(0): the reads above have completed */
            WAVE_SYNC();
#pragma unroll
            for (int r = 0; r < MAXR; ++r) {
                const int i = (r << 6) + lane;
                if (i < n) {
                    const int j = n - 1 - i;
                    const int2 x0 = U(s, 0, j), x1 = U(s, 1, j);
                    a.bk[FP][off + i] = x0.x; a.bk[FQ][off + i] = x0.y;
                    a.bk[FO][off + i] = x1.x; a.bk[FT][off + i] = x1.y;
                    a.bk[FS][off + i] = ts[r]; a.bk[FN][off + i] = tn[r];
                }
            }
            WAVE_SYNC();
        }
        if (lane == 0) {
            a.bk_n[gb] = n0;
            a.bk_n[gb + 1] = n1;
        }
        if (lane < ENVW) a.env_state[(int64_t)e * ENVW + lane] = ENV()[lane];
        if (lane < NCTR) a.counters[(int64_t)e * LOB_N_COUNTERS + lane] = ctr;
        if (lane < STW) a.stats[(int64_t)e * STW + lane] = X64(xl().st)[lane];
        if (lane < A * AGW) a.agent_state[(int64_t)e * A * AGW + lane] = AG(0)[lane];
        if (a.trade_cursor && lane == 0) a.trade_cursor[e] = tr_cur0 + tr_next;
    }

    /* The cancel block's walk for agent ai over side S: its resting orders in book order
     * (best first); an order at a level the agent no longer wants is deleted, at a kept
     * level any excess over the desired quantity comes from its newest orders there.  A
     * cancel at record j moves only records above j, so the walk continues below j. */
    /* order j of agent ai in the walk: a cancel message (delete, or partial cancel of the
     * excess) when due; a removal shifts the held indices above it */
    template <int S> __device__ __forceinline__ void walk_order(int ai, int nlv, int j) {
        const int4 rj = *RQ<S>(j);
        const int pr = uni(rj.x), qt = uni(rj.y), oid = uni(rj.z);
        const int l = find_level(ai, nlv, S, pr);
        const int D = l >= 0 ? rdlane(lv_d, l) : 0;
        int x = qt; /* quantity to cancel; qt = the whole order */
        if (D > 0) {
            const int R = rdlane(lv_r, l);
            const int older = rdlane(lv_seen, l);
            lv_seen += lane == l ? qt : 0;
            x = R > D ? min(max((R - D) - (R - older - qt), 0), qt) : 0;
        }
        if (x > 0) {
            const int k = D == 0 ? cancel<S, CX_DELETE>(qt, oid) : cancel<S, CX_PARTIAL>(x, oid);
            after_message();
            if (k >= 0) al_jt[S] -= (al_jt[S] >> 3) > k ? 8 : 0;
        }
    }
    template <int S> __device__ __forceinline__ void walk_side(int ai, int nlv, int tid) {
        uint64_t m = ballot(lane < min(al_n[S], WAVE) && (al_jt[S] & 7) == tid);
        while (m) {
            const int p = (int)__builtin_ctzll(m);
            m &= m - 1;
            walk_order<S>(ai, nlv, rdlane(al_jt[S], p) >> 3);
        }
        if (al_n[S] > WAVE) {
            /* below the held orders, by search (the held index is current) */
            int hi = (rdlane(al_jt[S], WAVE - 1) >> 3) - 1;
            for (;;) {
                const int j = find_top<S>(FT, hi, tid);
                if (j < 0) break;
                walk_order<S>(ai, nlv, j);
                hi = j - 1;
            }
        }
    }

    /* ---- one env-step (Sec. 4 steps 1-5) writing output slot s_idx ---- */
    __device__ __forceinline__ void step(int s_idx) {
        const int N = a.n_envs;
        mid_sum = vreg64(0); mid_n = vreg32(0); seq = 0; mid_at = 0;
        touch_changed();
        st_buy = 0; st_sell = 0; st_last = 0;
        tr_step0 = tr_next;
        if (lane < A * 4) FL(0)[lane] = 0;
        WAVE_SYNC();
        /* reference prices at step start; an empty side keeps its last known best */
        const int bb0 = n0 > 0 ? best0 : (int)uni64(ENV()[0]);
        const int ba0 = n1 > 0 ? best1 : (int)uni64(ENV()[1]);

        /* step 1 (from the book at step start): every agent's desired levels and new
         * orders, agents in index order */
        int nact = 0;
        lv_side = 0; lv_price = 0; lv_d = 0; lv_r = 0; lv_seen = 0; lv_n = 0;
        if (A > 0) {
            agent_scan<0>();
            agent_scan<1>();
        }
        /* random actions: lane i draws agent i's (the counter hash on the vector units) */
        const uint32_t ua = a.actions_in ? 0u
                                         : (uint32_t)(hash4(a.seed, DOM_ACTION, (uint64_t)e, (uint64_t)t, (uint64_t)lane) >> 32);
        for (int i = 0; i < A; ++i) {
            const int kind = (a.kinds >> (4 * i)) & 15;
            const int nacts = kind_actions(kind);
            int act;
            if (a.actions_in) {
                act = uni(a.actions_in[((int64_t)s_idx * A + i) * N + e]);
            } else {
                const uint32_t u = (uint32_t)rdlane((int)ua, i);
                act = (int)(((uint64_t)u * (uint64_t)nacts) >> 32);
            }
            if (a.actions_out && lane == 0) a.actions_out[((int64_t)s_idx * A + i) * N + e] = act;
            if (act < 0 || act >= nacts) act = 0;
            agent_start(i, act, bb0, ba0, nact);
        }
        /* step 2: shuffle the new orders by (32-bit counter hash, position) */
        if (nact > 0) {
            const uint32_t key = (uint32_t)(hash4(a.seed, DOM_SHUFFLE, (uint64_t)e, (uint64_t)t, (uint64_t)lane) >> 32);
            int rank = 0;
            for (int j = 0; j < nact; ++j) {
                const uint32_t kj = (uint32_t)rdlane((int)key, j);
                rank += (kj < key || (kj == key && j < lane)) ? 1 : 0;
            }
            if (lane < nact) X()[xl().perm + rank] = lane;
            WAVE_SYNC();
        }

        /* steps 3-4, in the order of Sec. 4 step 3.  First the cancel block: agents in
         * index order, each walking its resting orders on both sides (walk_side). */
        for (int ai = 0; ai < A; ++ai) {
            const int tid = ai + 1;
            const int nlv = rdlane(lv_n, ai);
            walk_side<0>(ai, nlv, tid);
            walk_side<1>(ai, nlv, tid);
        }

        /* then the shuffled new orders (staged as the first chunk) and the replayed
         * messages (64 per chunk), one process() each */
        const int64_t *row = a.m_off + (int64_t)e * (a.m_steps + 1);
        const int64_t lo = uni64(row[t]);
        const int nrep = (int)(uni64(row[t + 1]) - lo);
        Staged m;
        if (lane < nact) {
            const int32_t *x = X() + xl().act + X()[xl().perm + lane] * 8;
            m.c[0] = x[0]; m.c[1] = x[1]; m.c[2] = x[2]; m.c[3] = x[3]; m.c[4] = x[4]; m.c[5] = x[5];
        }
        int cnt = nact, cb = -WAVE; /* cb: first replayed message of the chunk */
        for (;;) {
            /* everything the chunk loaded has arrived before the first message is read
             * (so no per-message waits on it) */
            __builtin_amdgcn_s_waitcnt(0);
            m.c[0] = op_code(m.c[0], m.c[2]);
            for (m.j = 0; m.j < cnt; ++m.j) process(m);
            cb += WAVE;
            if (cb >= nrep) break;
            const int nx = cb + lane;
            if (nx < nrep) {
                const int64_t g = lo + nx;
                m.c[0] = a.m_ts[g]; m.c[1] = a.m_price[g]; m.c[2] = a.m_qty[g]; m.c[3] = a.m_oid[g];
                m.c[4] = a.m_tid[g]; m.c[5] = (int)(g - sbase); /* the time stays in the stream */
            }
            cnt = min(WAVE, nrep - cb);
        }
        /* the last processed time: agent messages carry the previous one, so it changes
         * only with a replayed message */
        if (nrep > 0) {
            const int64_t gl = lo + nrep - 1;
            last_tsec = uni(a.m_tsec[gl]);
            last_tns = uni(a.m_tns[gl]);
            last_ref = (int)(gl - sbase);
        }

        /* step 5: outcomes */
        mid_flush();
        int64_t *E = ENV();
        const int64_t mid2_prev = uni64(E[2]), p_init2 = uni64(E[3]);
        const int bb1 = n0 > 0 ? best0 : (int)uni64(E[0]);
        const int ba1 = n1 > 0 ? best1 : (int)uni64(E[1]);
        const int64_t mid2_end = (int64_t)bb1 + ba1;
        const bool last = (t + 1 == a.episode_len);
        const double mbar = mid_n > 0 ? (double)mid_sum / (2.0 * (double)mid_n) : (double)mid2_prev * 0.5;
        const double mt = (double)mid2_end * 0.5;
        const double mprev = (double)mid2_prev * 0.5;
        for (int i = 0; i < A; ++i) {
            const int kind = (a.kinds >> (4 * i)) & 15;
            const int64_t *fl = FL(i);
            const int64_t bq = uni64(fl[0]), bn = uni64(fl[1]), sq = uni64(fl[2]), sn = uni64(fl[3]);
            int64_t *g = AG(i);
            const int64_t inv = uni64(g[0]) + bq - sq;
            const int64_t cash = uni64(g[1]) + sn - bn;
            const int64_t rem = uni64(g[2]) - (exec_kind(kind) ? sq : 0);
            const double psi_b = mbar * (double)bq - (double)bn;
            const double psi_s = (double)sn - mbar * (double)sq;
            double r;
            if (spooner_kind(kind)) {
                /* Eq. 3 with the quadratic inventory penalty */
                const double psi_inv = (double)inv * (mt - mprev);
                const double pos = psi_inv > 0.0 ? psi_inv : 0.0;
                r = psi_b + psi_s + psi_inv - (1.0 - (double)a.lam) * pos - (double)a.rho * ((double)inv * (double)inv);
            } else if (kind == LOB_AGENT_MM_BUYSELL) {
                /* Eq. 4 with the quadratic inventory penalty */
                r = psi_b + psi_s - (double)a.rho * ((double)inv * (double)inv);
            } else if (kind == LOB_AGENT_DIR) {
                /* Eq. 4 */
                r = psi_b + psi_s;
            } else {
                /* Eq. 2 per step against the price at reset, with the end penalty */
                const double pinit = (double)p_init2 * 0.5;
                r = (double)sn - pinit * (double)sq;
                if (last) r = r - ((double)a.pen * (double)rem) * pinit;
            }
            if (lane == 0) {
                g[0] = inv; g[1] = cash; g[2] = rem; g[4] = bq; g[5] = sq;
                a.reward[((int64_t)s_idx * A + i) * N + e] = (float)r;
            }
            if (lane < 4) a.fills[(((int64_t)s_idx * A + i) * N + e) * 4 + lane] = fl[lane];
        }
        /* counters of the step; trade records beyond the env's region were not written */
        const int st_trades = tr_next - tr_step0;
        const int written_end = max(tr_step0, tr_room);
        const int overflow = tr_next > written_end ? tr_next - written_end : 0;
        count(C_MSGS, seq);
        count(C_TRADES, st_trades);
        count(C_TRADE_OVERFLOW, overflow);
        if (lane == 0) {
            int64_t *S = X64(xl().st);
            S[0] = st_buy; S[1] = st_sell; S[2] = st_trades; S[3] = st_last;
            E[0] = bb1; E[1] = ba1; E[2] = mid2_end; E[4] = last_tsec; E[5] = last_tns;
            E[6] = t + 1; E[7] = mid2_end - mid2_prev;
            a.n_trades[(int64_t)s_idx * N + e] = st_trades;
            a.done[(int64_t)s_idx * N + e] = last ? 1 : 0;
        }
        WAVE_SYNC();
        t += 1;
        if (a.obs) write_obs(a.obs + (int64_t)s_idx * A * N * LOB_OBS_DIM);
    }
};

/* ------------------------------------------------------------------------------
 * Kernels
 * ---------------------------------------------------------------------------- */
/* 256 threads, at least 4 waves per SIMD: up to 128 VGPRs (it takes 110, no spills).
 * LDS, not registers, bounds the resident envs of the large books; capping registers at
 * 80 for 6 waves per SIMD spilled to scratch and was 2% slower on the uneven workload. */
__global__ void __launch_bounds__(256, 4) k_env(KArgs a) {
    extern __shared__ int32_t smem[];
    const int wave = uni((int)(threadIdx.x >> 6)), waves = (int)(blockDim.x >> 6);
    int32_t *L = smem + wave * a.lds_words;
    for (;;) {
        int slot;
        if (a.work_ctr) {
            int v = 0;
            if (lane_id() == 0) v = atomicAdd(a.work_ctr, 1);
            slot = rdlane(v, 0);
        } else {
            slot = (int)blockIdx.x * waves + wave;
        }
        if (slot >= a.n_list) break;
        Run run(a, L, a.env_list[slot]);
        run.load();
        for (int s = 0; s < a.n_steps; ++s) run.step(s);
        run.store();
        if (!a.work_ctr) break;
    }
}

/* observation of the current state (no step) */
__global__ void __launch_bounds__(256) k_observe(KArgs a) {
    extern __shared__ int32_t smem[];
    const int wave = uni((int)(threadIdx.x >> 6)), waves = (int)(blockDim.x >> 6);
    const int slot = (int)blockIdx.x * waves + wave;
    if (slot >= a.n_list) return;
    int32_t *L = smem + wave * a.lds_words;
    Run run(a, L, a.env_list[slot]);
    run.load();
    run.write_obs(a.obs);
}

struct ResetArgs {
    int32_t n_envs, n_agents, max_cap, kinds, exec_task;
    const int32_t *caps;
    const int32_t *src[NF];
    const int32_t *src_n;
    int32_t *dst[NF];
    int32_t *dst_n;
    int64_t *env_state, *agent_state, *counters, *stats;
};

__global__ void __launch_bounds__(256) k_reset(ResetArgs a) {
    const int wave = (int)(threadIdx.x >> 6), waves = (int)(blockDim.x >> 6);
    const int e = (int)blockIdx.x * waves + wave;
    if (e >= a.n_envs) return;
    const int lane = lane_id();
    const int cap = a.caps[e];
    int n[2];
    int64_t tkey = 0x80000000ll; /* time (0, 0): tsec << 32 | (tns ^ 0x80000000) */
    for (int s = 0; s < 2; ++s) {
        n[s] = min(max(uni(a.src_n[e * 2 + s]), 0), cap);
        const int64_t off = ((int64_t)e * 2 + s) * a.max_cap;
        for (int i = lane; i < n[s]; i += WAVE) {
#pragma unroll
            for (int f = 0; f < NF; ++f) a.dst[f][off + i] = a.src[f][off + i];
            const int64_t k = ((int64_t)a.src[FS][off + i] << 32) | (int64_t)(uint32_t)(a.src[FN][off + i] ^ (int)0x80000000);
            tkey = max(tkey, k);
        }
        if (lane == 0) a.dst_n[e * 2 + s] = n[s];
    }
#pragma unroll
    for (int d = WAVE / 2; d >= 1; d >>= 1) tkey = max(tkey, (int64_t)__shfl_xor(tkey, d, WAVE));
    const int64_t off0 = (int64_t)e * 2 * a.max_cap, off1 = ((int64_t)e * 2 + 1) * a.max_cap;
    const int bp = n[0] > 0 ? uni(a.src[FP][off0]) : 0;
    const int ap = n[1] > 0 ? uni(a.src[FP][off1]) : 0;
    const int bb = n[0] > 0 ? bp : (n[1] > 0 ? ap - 1 : 0);
    const int ba = n[1] > 0 ? ap : (n[0] > 0 ? bp + 1 : 0);
    const int64_t m2 = (int64_t)bb + ba;
    int64_t v = 0;
    switch (lane) {
    case 0: v = bb; break;
    case 1: v = ba; break;
    case 2: v = m2; break;
    case 3: v = m2; break;
    case 4: v = (int32_t)(tkey >> 32); break;
    case 5: v = (int32_t)((uint32_t)tkey ^ 0x80000000u); break;
    default: v = 0; break;
    }
    if (lane < ENVW) a.env_state[(int64_t)e * ENVW + lane] = v;
    if (lane < LOB_N_COUNTERS) a.counters[(int64_t)e * LOB_N_COUNTERS + lane] = 0;
    if (lane < STW) a.stats[(int64_t)e * STW + lane] = 0;
    if (lane < a.n_agents * AGW) {
        const int i = lane / AGW, w = lane % AGW;
        const int kind = (a.kinds >> (4 * i)) & 15;
        a.agent_state[(int64_t)e * a.n_agents * AGW + lane] = (w == 2 && exec_kind(kind)) ? (int64_t)a.exec_task : 0;
    }
}

struct ExportArgs {
    int32_t n_envs, n_agents, max_cap;
    const int32_t *src[NF];
    const int32_t *src_n;
    int32_t *dst[NF];
    int32_t *dst_n;
    const int64_t *agent_src;
    int64_t *agent_dst;
    const int64_t *env_src, *stats_src;
    int64_t *env_dst;
};

__global__ void k_export_books(ExportArgs a) {
    const int64_t total = (int64_t)a.n_envs * 2 * a.max_cap;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
        const int64_t es = g / a.max_cap;
        const int i = (int)(g - es * a.max_cap);
        const bool live = i < a.src_n[es];
#pragma unroll
        for (int f = 0; f < NF; ++f) a.dst[f][g] = live ? a.src[f][g] : 0;
        if (i == 0) a.dst_n[es] = a.src_n[es];
    }
}

__global__ void k_export_agents(ExportArgs a) {
    const int64_t total = (int64_t)a.n_envs * a.n_agents * LOB_AGENT_STATE_WORDS;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
        const int64_t ea = g / LOB_AGENT_STATE_WORDS;
        const int w = (int)(g - ea * LOB_AGENT_STATE_WORDS);
        a.agent_dst[g] = a.agent_src[ea * AGW + w];
    }
}

/* exported env state: the internal words, then the last step's statistics */
__global__ void k_export_env(ExportArgs a) {
    const int64_t total = (int64_t)a.n_envs * LOB_ENV_STATE_WORDS;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = g / LOB_ENV_STATE_WORDS;
        const int w = (int)(g - e * LOB_ENV_STATE_WORDS);
        a.env_dst[g] = w < ENVW ? a.env_src[e * ENVW + w] : a.stats_src[e * STW + (w - ENVW)];
    }
}

/* The inverse of the exports: books in canonical layout (counts clamped to each env's
 * capacity, unused slots ignored) and the exported state, with every env's step counter
 * set to `step`; counters may be absent (zero). */
struct ImportArgs {
    int32_t n_envs, n_agents, max_cap, step;
    const int32_t *caps;
    const int32_t *src[NF];
    const int32_t *src_n;
    const int64_t *env_src, *agent_src, *ctr_src;
    int32_t *dst[NF];
    int32_t *dst_n;
    int64_t *env_state, *agent_state, *counters, *stats;
};

__global__ void __launch_bounds__(256) k_import(ImportArgs a) {
    const int wave = (int)(threadIdx.x >> 6), waves = (int)(blockDim.x >> 6);
    const int e = (int)blockIdx.x * waves + wave;
    if (e >= a.n_envs) return;
    const int lane = lane_id();
    const int cap = a.caps[e];
    for (int s = 0; s < 2; ++s) {
        const int n = min(max(a.src_n[e * 2 + s], 0), cap);
        const int64_t off = ((int64_t)e * 2 + s) * a.max_cap;
        for (int i = lane; i < n; i += WAVE) {
#pragma unroll
            for (int f = 0; f < NF; ++f) a.dst[f][off + i] = a.src[f][off + i];
        }
        if (lane == 0) a.dst_n[e * 2 + s] = n;
    }
    const int64_t *es = a.env_src + (int64_t)e * LOB_ENV_STATE_WORDS;
    if (lane < ENVW) a.env_state[(int64_t)e * ENVW + lane] = lane == 6 ? (int64_t)a.step : es[lane];
    if (lane < STW) a.stats[(int64_t)e * STW + lane] = es[ENVW + lane];
    if (lane < NCTR) a.counters[(int64_t)e * LOB_N_COUNTERS + lane] = a.ctr_src ? a.ctr_src[(int64_t)e * LOB_N_COUNTERS + lane] : 0;
    if (lane < a.n_agents * AGW) {
        const int i = lane / AGW, w = lane % AGW;
        a.agent_state[(int64_t)e * a.n_agents * AGW + lane] =
            w < LOB_AGENT_STATE_WORDS ? a.agent_src[((int64_t)e * a.n_agents + i) * LOB_AGENT_STATE_WORDS + w] : 0;
    }
}

/* Holds its stream for `ticks` of the constant-rate wall clock (one wave, sleeping
 * between reads: the wait is bounded by the clock). */
__global__ void k_hold(int64_t ticks) {
    const int64_t t0 = (int64_t)wall_clock64();
    while ((int64_t)wall_clock64() - t0 < ticks) __builtin_amdgcn_s_sleep(16);
}

__global__ void k_fill_i32(int32_t *p, int32_t n, int32_t v) {
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < n) p[i] = v;
}

} // namespace lobk

/* ==================================================================================
 * Host side: the C-ABI
 * ================================================================================ */
using namespace lobk;

struct CapClass {
    int rows;      /* rows of 64 records a book of the class spans */
    int capp;      /* records per side in LDS: the largest capacity in the class */
    int first;     /* offset into the env list */
    int count;     /* envs in the class */
    int waves;     /* waves per workgroup (one env per wave) */
    int mode;      /* 0: one wave per env, hardware dispatch in list order; 1: work queue */
    int grid;      /* workgroups in queue mode (0 = derived from occupancy) */
};

constexpr int MAX_CLASSES = LOB_MAX_CAP / 64; /* one class per row count */
constexpr size_t LDS_PER_CU = 160 * 1024;  /* gfx950 */
constexpr int64_t LANE_GAP_US = 50;      /* between class starts in a rollout */
constexpr int64_t LANE_GAP_STEP_US = 10; /* between class starts in a one-step launch */
constexpr int CONC_LANES = 3;               /* concurrent class launches (see launch_env) */
constexpr int WAVES_PER_CU = 16;            /* 4 per SIMD at the env kernel's register use */
constexpr int BALANCE_DEFAULT = 880;        /* permille of the LDS (measured best on uneven books) */
constexpr int64_t STEP_ALLOWANCE = 8;       /* fixed per-env-step work, in messages */

struct lob_ctx {
    lob_config cfg;
    std::vector<int32_t> caps, kinds;
    int32_t kinds_packed = 0;
    double avst[18] = {};            /* Avellaneda-Stoikov quote terms per risk-aversion choice */
    double *d_avst = nullptr;        /* the same on the device */
    int32_t *d_caps = nullptr;
    int32_t *d_bk[NF] = {};
    int32_t *d_bk_n = nullptr;
    int64_t *d_env = nullptr, *d_agent = nullptr, *d_ctr = nullptr, *d_stats = nullptr;
    int32_t *d_env_list = nullptr;  /* envs grouped by class, each class longest first */
    int32_t *d_work = nullptr;      /* work-queue counters, one per class */
    std::vector<int32_t> env_list;  /* host copy */
    std::vector<CapClass> classes;
    hipStream_t streams[MAX_CLASSES] = {};
    hipEvent_t ev_fork = nullptr, ev_join[MAX_CLASSES] = {};
    /* recorded on the caller's stream after each launch (lanes joined): the host waits
     * for it before rewriting what running launches read (env list, work queues) */
    hipEvent_t ev_done = nullptr;
    bool launched = false, captured = false;
    /* the plan: which (stream offsets, first step, steps) the env order was made for */
    const int64_t *plan_off = nullptr;
    int64_t plan_n_msgs = -1;
    int plan_t0 = -1, plan_steps = -1, plan_rows = -1;
    int device = 0;
    int n_cu = 256;
    int64_t ticks_per_us = 100; /* of the device's wall clock (its rate is read at init) */
    int t = 0;
    bool reset_done = false;
    bool padded = false;
    /* with several classes, the share of the chip's LDS (permille) that the proportional
     * work-queue schedule gives the classes together; 0 = each class keeps its own
     * schedule (see balance_classes) */
    int balance = BALANCE_DEFAULT;
};

namespace {

bool hip_ok(hipError_t e) { return e == hipSuccess; }

template <class T>
int dalloc(T **p, size_t n) {
    if (n == 0) n = 1;
    if (hipMalloc(reinterpret_cast<void **>(p), n * sizeof(T)) != hipSuccess) {
        *p = nullptr;
        return LOB_ENOMEM;
    }
    return LOB_OK;
}

void free_ctx(lob_ctx *c) {
    if (!c) return;
    (void)hipFree(c->d_caps);
    for (int f = 0; f < NF; ++f) (void)hipFree(c->d_bk[f]);
    (void)hipFree(c->d_bk_n);
    (void)hipFree(c->d_env);
    (void)hipFree(c->d_agent);
    (void)hipFree(c->d_ctr);
    (void)hipFree(c->d_stats);
    (void)hipFree(c->d_env_list);
    (void)hipFree(c->d_work);
    (void)hipFree(c->d_avst);
    for (int k = 0; k < MAX_CLASSES; ++k) {
        if (c->streams[k]) (void)hipStreamDestroy(c->streams[k]);
        if (c->ev_join[k]) (void)hipEventDestroy(c->ev_join[k]);
    }
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_done) (void)hipEventDestroy(c->ev_done);
    delete c;
}

KArgs base_args(const lob_ctx *c) {
    KArgs a;
    std::memset(&a, 0, sizeof(a));
    a.n_envs = c->cfg.n_envs;
    a.n_agents = c->cfg.n_agents;
    a.max_cap = c->cfg.max_cap;
    a.episode_len = c->cfg.episode_len;
    a.seed = c->cfg.seed;
    a.exec_task = c->cfg.exec_task;
    a.exec_q0 = c->cfg.exec_q0;
    a.mm_q = c->cfg.mm_q;
    a.dir_q = c->cfg.dir_q;
    a.pen = c->cfg.exec_penalty;
    a.lam = c->cfg.mm_lambda;
    a.rho = c->cfg.mm_rho;
    a.avst = c->d_avst;
    a.kinds = c->kinds_packed;
    a.caps = c->d_caps;
    for (int f = 0; f < NF; ++f) a.bk[f] = c->d_bk[f];
    a.bk_n = c->d_bk_n;
    a.env_state = c->d_env;
    a.agent_state = c->d_agent;
    a.counters = c->d_ctr;
    a.stats = c->d_stats;
    return a;
}

int check_msgs(const lob_ctx *c, const lob_msgs *m, int n_steps) {
    if (!m || !m->ts || !m->price || !m->qty || !m->oid || !m->tid || !m->tsec || !m->tns || !m->off)
        return LOB_EINVAL;
    if (m->n_steps < 0 || m->n_msgs < 0) return LOB_EINVAL;
    if (c->t + n_steps > m->n_steps) return LOB_ESTATE;
    return LOB_OK;
}

int check_out(const lob_ctx *c, const lob_out *o) {
    if (!o || !o->n_trades || !o->done) return LOB_EINVAL;
    if (c->cfg.n_agents > 0 && (!o->fills || !o->reward)) return LOB_EINVAL;
    if (o->trades && !o->trade_off) return LOB_EINVAL;
    return LOB_OK;
}

void fill_msgs(KArgs &a, const lob_msgs *m) {
    a.m_ts = m->ts; a.m_price = m->price; a.m_qty = m->qty; a.m_oid = m->oid;
    a.m_tid = m->tid; a.m_tsec = m->tsec; a.m_tns = m->tns;
    a.m_off = m->off; a.m_steps = m->n_steps;
}

void fill_out(KArgs &a, const lob_out *o) {
    a.trades = o->trades; a.trade_off = o->trade_off; a.trade_cursor = o->trade_cursor;
    a.n_trades = o->n_trades; a.fills = o->fills; a.reward = o->reward; a.obs = o->obs;
    a.done = o->done; a.actions_out = o->actions;
}

size_t class_lds(const lob_ctx *c, const CapClass &cl) {
    return (size_t)lds_words_for(cl.capp, c->cfg.n_agents) * 4 * cl.waves;
}

/* Launch the env kernel of one class on stream st. */
int launch_class(lob_ctx *c, size_t k, KArgs a, hipStream_t st) {
    const CapClass &cl = c->classes[k];
    if (cl.count == 0) return LOB_OK;
    a.capp = cl.capp;
    a.lds_words = lds_words_for(cl.capp, c->cfg.n_agents);
    a.env_list = c->d_env_list + cl.first;
    a.n_list = cl.count;
    const int waves = cl.waves;
    const size_t lds = class_lds(c, cl);
    int grid;
    if (cl.mode == 1) {
        a.work_ctr = c->d_work + k;
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, c->d_work + k, 1, 0);
        int per_cu = (int)(LDS_PER_CU / lds);
        if (per_cu < 1) per_cu = 1;
        grid = cl.grid > 0 ? cl.grid : c->n_cu * per_cu;
        grid = std::min(grid, (cl.count + waves - 1) / waves);
    } else {
        a.work_ctr = nullptr;
        grid = (cl.count + waves - 1) / waves;
    }
    hipLaunchKernelGGL(k_env, dim3(grid), dim3(64 * waves), lds, st, a);
    return hipGetLastError() == hipSuccess ? LOB_OK : LOB_EHIP;
}

/* Launch every class concurrently: lane 0 is the caller's stream, lanes 1.. are forked
 * streams joined back with events.  A process has few hardware queues (4 by default, one
 * of them taken by other work in practice) and streams beyond them share queues,
 * serialising their kernels; so there are at most CONC_LANES lanes, and classes are
 * merged to at most that many (build_classes).  Classes are dealt to the lanes largest
 * books first; classes sharing a lane would run one after the other. */
int launch_env(lob_ctx *c, KArgs a, hipStream_t st) {
    const int nc = (int)c->classes.size();
    const int lanes = std::min(nc, CONC_LANES);
    if (lanes > 1 && !hip_ok(hipEventRecord(c->ev_fork, st))) return LOB_EHIP;
    /* lanes forked from the caller's stream so far: every one of them is joined back
     * below, also when a launch fails (an unjoined fork would invalidate a stream
     * capture, and the caller's stream would not wait for work already queued) */
    int forked = 1, rc = LOB_OK;
    for (int l = 1; l < lanes && rc == LOB_OK; ++l) {
        if (!hip_ok(hipStreamWaitEvent(c->streams[l], c->ev_fork, 0))) {
            rc = LOB_EHIP;
            break;
        }
        forked = l + 1;
        /* The classes start one after another, largest books first, LANE_GAP_US apart (a
         * single step: LANE_GAP_STEP_US, which it pays every step): started at the same
         * instant, the workgroups of two classes interleave differently from run to run,
         * and one of them could be left slower than planned for the whole launch (3 us
         * apart still did; smallest books first took twice as long: the large workgroups
         * then find no room). */
        hipLaunchKernelGGL(k_hold, dim3(1), dim3(64), 0, c->streams[l],
                           (int64_t)((a.n_steps > 1 ? LANE_GAP_US : LANE_GAP_STEP_US) * c->ticks_per_us * l));
        if (hipGetLastError() != hipSuccess) rc = LOB_EHIP;
    }
    for (int i = 0; i < nc && rc == LOB_OK; ++i) {
        const int k = nc - 1 - i; /* largest books first */
        const int l = i % lanes;
        rc = launch_class(c, (size_t)k, a, l == 0 ? st : c->streams[l]);
    }
    for (int l = 1; l < forked; ++l) {
        if (!hip_ok(hipEventRecord(c->ev_join[l], c->streams[l])) ||
            !hip_ok(hipStreamWaitEvent(st, c->ev_join[l], 0)))
            rc = rc != LOB_OK ? rc : LOB_EHIP;
    }
    /* under stream capture the launch runs when the graph is replayed, which this
     * context does not see: later waits fall back to the whole device */
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hip_ok(hipStreamIsCapturing(st, &cs)) && cs == hipStreamCaptureStatusNone) {
        if (!hip_ok(hipEventRecord(c->ev_done, st))) rc = rc != LOB_OK ? rc : LOB_EHIP;
        c->launched = true;
    } else {
        c->captured = true;
    }
    return rc;
}

/* Wait until no launch of this context can still be running: the last eager launch's
 * completion event, or the whole device once a launch was captured into a graph. */
bool wait_launches(lob_ctx *c) {
    if (c->captured) return hip_ok(hipDeviceSynchronize());
    return !c->launched || hip_ok(hipEventSynchronize(c->ev_done));
}

/* Default waves (envs) per workgroup for a class: the most resident envs per CU, LDS
 * being allocated per workgroup (at most 64 KiB each); ties go to larger workgroups. */
int default_waves(int capp, int n_agents) {
    const size_t per_wave = (size_t)lds_words_for(capp, n_agents) * 4;
    int best_w = 1, best_n = -1;
    for (int w : {4, 2, 1}) {
        if (per_wave * w > 64 * 1024) continue;
        const int n = std::min((int)(LDS_PER_CU / (per_wave * w)) * w, WAVES_PER_CU / w * w);
        if (n > best_n) { best_n = n; best_w = w; }
    }
    return best_w;
}

/* Group the envs into capacity classes: envs whose books span the same number of rows
 * share a class whose LDS books are sized for the largest capacity among them; with
 * `padded` every env goes into one class sized for the largest capacity overall.  Envs
 * are listed in index order until a plan orders them; streams and events for the
 * classes' concurrent launches are created on first use.  Host-synchronous. */
int build_classes(lob_ctx *c, bool padded) {
    const int N = c->cfg.n_envs;
    std::vector<int> rows;
    for (int32_t v : c->caps) rows.push_back(padded ? 0 : rows_for_cap(v));
    std::vector<int> uniq(rows);
    std::sort(uniq.begin(), uniq.end());
    uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
    if (uniq.size() > (size_t)MAX_CLASSES) return LOB_EUNSUPPORTED;
    /* groups of row counts: start with one group per row count, then merge the adjacent
     * pair whose merge adds the least LDS (the smaller group's envs sized for the larger
     * capacity) until at most CONC_LANES groups remain, so every class runs concurrently */
    struct Grp { int lo, hi, count, capp; };
    std::vector<Grp> g;
    for (int r : uniq) {
        Grp x{r, r, 0, 0};
        for (int e = 0; e < N; ++e)
            if (rows[(size_t)e] == r) { x.count++; x.capp = std::max(x.capp, c->caps[(size_t)e]); }
        g.push_back(x);
    }
    const int A = c->cfg.n_agents;
    while ((int)g.size() > CONC_LANES) {
        size_t bi = 0;
        int64_t bcost = -1;
        for (size_t i = 0; i + 1 < g.size(); ++i) {
            const int64_t cost = (int64_t)g[i].count * (lds_words_for(g[i + 1].capp, A) - lds_words_for(g[i].capp, A));
            if (bcost < 0 || cost < bcost) { bcost = cost; bi = i; }
        }
        g[bi + 1].lo = g[bi].lo;
        g[bi + 1].count += g[bi].count;
        g.erase(g.begin() + (std::ptrdiff_t)bi);
    }
    c->classes.clear();
    c->env_list.clear();
    for (const Grp &x : g) {
        CapClass cl{0, 0, (int)c->env_list.size(), 0, 1, 0, 0};
        for (int e = 0; e < N; ++e)
            if (rows[(size_t)e] >= x.lo && rows[(size_t)e] <= x.hi) {
                c->env_list.push_back(e);
                cl.count++;
                cl.capp = std::max(cl.capp, c->caps[(size_t)e]);
            }
        cl.rows = rows_for_cap(cl.capp);
        cl.waves = default_waves(cl.capp, A);
        c->classes.push_back(cl);
    }
    for (size_t k = 0; k < c->classes.size(); ++k) {
        if (!c->streams[k] && !hip_ok(hipStreamCreateWithFlags(&c->streams[k], hipStreamNonBlocking)))
            return LOB_EHIP;
        if (!c->ev_join[k] && !hip_ok(hipEventCreateWithFlags(&c->ev_join[k], hipEventDisableTiming)))
            return LOB_EHIP;
    }
    c->plan_off = nullptr;
    c->plan_t0 = c->plan_steps = -1;
    c->padded = padded;
    if (!hip_ok(hipMemcpy(c->d_env_list, c->env_list.data(), (size_t)N * 4, hipMemcpyHostToDevice)))
        return LOB_EHIP;
    return LOB_OK;
}

/* Proportional work-queue schedule for several concurrent classes.  Left to the hardware
 * dispatcher, the classes' workgroups compete for LDS as it frees and one class can be
 * starved for most of the run, its long envs then forming a tail.  Instead each class
 * runs as a work queue (mode 1) whose resident envs are proportional to the class's
 * work, so that the classes finish together: work = planned messages plus a fixed
 * allowance per env-step, and the classes together take `balance` permille of the
 * chip's LDS (below 1000 to leave room for packing workgroups of different sizes). */
void balance_classes(lob_ctx *c, const std::vector<int64_t> &a0, const std::vector<int64_t> &a1, int n) {
    const int A = c->cfg.n_agents;
    const size_t nc = c->classes.size();
    std::vector<double> work(nc, 0.0);
    double denom = 0.0;
    for (size_t k = 0; k < nc; ++k) {
        const CapClass &cl = c->classes[k];
        for (int i = 0; i < cl.count; ++i) {
            const size_t e = (size_t)c->env_list[(size_t)(cl.first + i)];
            work[k] += (double)(a1[e] - a0[e] + STEP_ALLOWANCE * n);
        }
        denom += work[k] * (double)lds_words_for(cl.capp, A) * 4.0;
    }
    const double budget = (double)c->balance / 1000.0 * (double)LDS_PER_CU * (double)c->n_cu;
    for (size_t k = 0; k < nc; ++k) {
        CapClass &cl = c->classes[k];
        cl.waves = default_waves(cl.capp, A);
        const int most = (cl.count + cl.waves - 1) / cl.waves;
        const double envs = denom > 0.0 ? budget * work[k] / denom : (double)cl.count;
        cl.mode = 1;
        cl.grid = std::max(1, std::min(most, (int)std::ceil(envs / cl.waves)));
    }
}

/* Order each class's envs by decreasing message count over steps [t0, t0+n) (longest
 * first), so the envs that bound the runtime start first; with several classes and a
 * balance share set, size their work queues (balance_classes).  Reads two columns of
 * the CSR offsets back to the host (synchronous). */
int make_plan(lob_ctx *c, const lob_msgs *m, int t0, int n) {
    /* the plan is kept while the stream (offsets array, its size and step rows) and the
     * steps are the same */
    if (c->plan_off == m->off && c->plan_n_msgs == m->n_msgs && c->plan_rows == m->n_steps && c->plan_t0 == t0 &&
        c->plan_steps == n)
        return LOB_OK;
    /* a launch still running (on the caller's stream or the class streams, which do not
     * synchronise with the null stream) may be reading the env list and the schedule
     * about to be rewritten: wait for it first */
    if (!wait_launches(c)) return LOB_EHIP;
    const int N = c->cfg.n_envs;
    const size_t pitch = (size_t)(m->n_steps + 1) * sizeof(int64_t);
    std::vector<int64_t> a0((size_t)N), a1((size_t)N);
    if (!hip_ok(hipMemcpy2D(a0.data(), 8, m->off + t0, pitch, 8, (size_t)N, hipMemcpyDeviceToHost)) ||
        !hip_ok(hipMemcpy2D(a1.data(), 8, m->off + t0 + n, pitch, 8, (size_t)N, hipMemcpyDeviceToHost)))
        return LOB_EHIP;
    for (const CapClass &cl : c->classes) {
        auto b = c->env_list.begin() + cl.first;
        std::stable_sort(b, b + cl.count, [&](int32_t x, int32_t y) {
            return a1[(size_t)x] - a0[(size_t)x] > a1[(size_t)y] - a0[(size_t)y];
        });
    }
    if (c->balance > 0 && c->classes.size() > 1) balance_classes(c, a0, a1, n);
    if (!hip_ok(hipMemcpy(c->d_env_list, c->env_list.data(), (size_t)N * 4, hipMemcpyHostToDevice)))
        return LOB_EHIP;
    c->plan_off = m->off;
    c->plan_n_msgs = m->n_msgs;
    c->plan_rows = m->n_steps;
    c->plan_t0 = t0;
    c->plan_steps = n;
    return LOB_OK;
}

} // namespace

extern "C" {

const char *lob_strerror(int code) {
    switch (code) {
    case LOB_OK: return "ok";
    case LOB_EINVAL: return "invalid argument";
    case LOB_ENOMEM: return "device allocation failed";
    case LOB_EHIP: return "HIP runtime error";
    case LOB_ESTATE: return "call out of order (not reset, episode over, or stream exhausted)";
    case LOB_EUNSUPPORTED: return "unsupported configuration";
    default: return "unknown error";
    }
}

int lob_init(const lob_config *cfg, lob_ctx **out) {
    if (!cfg || !out) return LOB_EINVAL;
    *out = nullptr;
    if (cfg->n_envs <= 0 || cfg->n_agents < 0 || cfg->n_agents > LOB_MAX_AGENTS || cfg->max_cap <= 0 ||
        cfg->episode_len <= 0 || !cfg->cap || (cfg->n_agents > 0 && !cfg->agent_kind) || cfg->flags != 0)
        return LOB_EINVAL;
    if (cfg->max_cap > LOB_MAX_CAP) return LOB_EUNSUPPORTED;
    if (cfg->exec_q0 < 0 || cfg->mm_q < 0 || cfg->dir_q < 0 || cfg->exec_task < 0) return LOB_EINVAL;
    lob_ctx *c = new (std::nothrow) lob_ctx();
    if (!c) return LOB_ENOMEM;
    c->cfg = *cfg;
    c->caps.assign(cfg->cap, cfg->cap + cfg->n_envs);
    for (int32_t v : c->caps)
        if (v < 1 || v > cfg->max_cap) { delete c; return LOB_EINVAL; }
    for (int i = 0; i < cfg->n_agents; ++i) {
        const int k = cfg->agent_kind[i];
        if (k < 0 || k > LOB_AGENT_MM_AS) { delete c; return LOB_EINVAL; }
        c->kinds.push_back(k);
        c->kinds_packed |= k << (4 * i);
    }
    bool avst = false;
    for (int32_t k : c->kinds) avst = avst || k == LOB_AGENT_MM_AVST || k == LOB_AGENT_MM_AS;
    if (avst) {
        /* Avellaneda-Stoikov quotes: gamma0 > 0, kappa > 0, sigma^2 >= 0 (finite), quotes of
         * mm_q > 0; the choice g takes gamma = gamma0 2^(g - 4) */
        const float g0 = cfg->avst_gamma, s2 = cfg->avst_sigma2, kp = cfg->avst_kappa;
        if (!(g0 > 0.f && kp > 0.f && s2 >= 0.f && std::isfinite(g0) && std::isfinite(kp) && std::isfinite(s2) &&
              cfg->mm_q > 0)) {
            delete c;
            return LOB_EINVAL;
        }
        for (int g = 0; g < 9; ++g) {
            const double gamma = (double)g0 * std::ldexp(1.0, g - 4);
            c->avst[g] = gamma * (double)s2;
            c->avst[9 + g] = (2.0 / gamma) * std::log(1.0 + gamma / (double)kp);
        }
    }
    c->cfg.cap = nullptr;
    c->cfg.agent_kind = nullptr;
    if (!hip_ok(hipGetDevice(&c->device))) { delete c; return LOB_EHIP; }
    hipDeviceProp_t prop;
    if (hip_ok(hipGetDeviceProperties(&prop, c->device))) c->n_cu = prop.multiProcessorCount;
    /* the wall clock's rate differs between boxes (100 MHz on some, 30 MHz on others): the
     * class-start gaps are set in microseconds */
    int wall_khz = 0;
    if (hip_ok(hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, c->device)) && wall_khz >= 1000)
        c->ticks_per_us = wall_khz / 1000;

    const int64_t N = cfg->n_envs, A = cfg->n_agents;
    const size_t slots = (size_t)N * 2 * cfg->max_cap;
    int rc = LOB_OK;
    rc |= dalloc(&c->d_caps, (size_t)N);
    for (int f = 0; f < NF; ++f) rc |= dalloc(&c->d_bk[f], slots);
    rc |= dalloc(&c->d_bk_n, (size_t)N * 2);
    rc |= dalloc(&c->d_env, (size_t)N * ENVW);
    rc |= dalloc(&c->d_agent, (size_t)(N * std::max<int64_t>(A, 1) * AGW));
    rc |= dalloc(&c->d_ctr, (size_t)N * LOB_N_COUNTERS);
    rc |= dalloc(&c->d_stats, (size_t)N * STW);
    rc |= dalloc(&c->d_env_list, (size_t)N);
    rc |= dalloc(&c->d_work, 64);
    rc |= dalloc(&c->d_avst, 18);
    if (rc != LOB_OK) { free_ctx(c); return LOB_ENOMEM; }

    if ((rc = build_classes(c, false)) != LOB_OK) { free_ctx(c); return rc; }
    if (!hip_ok(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming)) ||
        !hip_ok(hipEventCreateWithFlags(&c->ev_done, hipEventDisableTiming)) ||
        !hip_ok(hipMemcpy(c->d_caps, c->caps.data(), (size_t)N * 4, hipMemcpyHostToDevice)) ||
        !hip_ok(hipMemcpy(c->d_avst, c->avst, sizeof(c->avst), hipMemcpyHostToDevice))) {
        free_ctx(c);
        return LOB_EHIP;
    }
    *out = c;
    return LOB_OK;
}

int lob_destroy(lob_ctx *c) {
    if (!c) return LOB_OK;
    (void)hipDeviceSynchronize();
    free_ctx(c);
    return LOB_OK;
}

int lob_current_step(const lob_ctx *c) { return c ? c->t : LOB_EINVAL; }

int lob_reset(lob_ctx *c, const lob_books *snap, void *stream) {
    if (!c || !snap || !snap->price || !snap->qty || !snap->oid || !snap->tid || !snap->tsec || !snap->tns || !snap->n)
        return LOB_EINVAL;
    ResetArgs a;
    std::memset(&a, 0, sizeof(a));
    a.n_envs = c->cfg.n_envs;
    a.n_agents = c->cfg.n_agents;
    a.max_cap = c->cfg.max_cap;
    a.kinds = c->kinds_packed;
    a.exec_task = c->cfg.exec_task;
    a.caps = c->d_caps;
    const int32_t *src[NF] = {snap->price, snap->qty, snap->oid, snap->tid, snap->tsec, snap->tns};
    for (int f = 0; f < NF; ++f) { a.src[f] = src[f]; a.dst[f] = c->d_bk[f]; }
    a.src_n = snap->n;
    a.dst_n = c->d_bk_n;
    a.env_state = c->d_env;
    a.agent_state = c->d_agent;
    a.counters = c->d_ctr;
    a.stats = c->d_stats;
    const int waves = 4;
    hipLaunchKernelGGL(k_reset, dim3((c->cfg.n_envs + waves - 1) / waves), dim3(64 * waves), 0,
                       (hipStream_t)stream, a);
    if (hipGetLastError() != hipSuccess) return LOB_EHIP;
    c->t = 0;
    c->reset_done = true;
    return LOB_OK;
}

int lob_step(lob_ctx *c, const lob_msgs *m, const int32_t *actions, const lob_out *o, void *stream) {
    if (!c) return LOB_EINVAL;
    if (!c->reset_done || c->t >= c->cfg.episode_len) return LOB_ESTATE;
    int rc = check_msgs(c, m, 1);
    if (rc != LOB_OK) return rc;
    if ((rc = check_out(c, o)) != LOB_OK) return rc;
    KArgs a = base_args(c);
    fill_msgs(a, m);
    fill_out(a, o);
    a.actions_in = actions;
    a.t0 = c->t;
    a.n_steps = 1;
    rc = launch_env(c, a, (hipStream_t)stream);
    if (rc != LOB_OK) return rc;
    c->t += 1;
    return LOB_OK;
}

int lob_rollout(lob_ctx *c, const lob_msgs *m, int32_t n_steps, const int32_t *actions, const lob_out *o,
                void *stream) {
    if (!c || n_steps < 0) return LOB_EINVAL;
    if (!c->reset_done || c->t + n_steps > c->cfg.episode_len) return LOB_ESTATE;
    if (n_steps == 0) return LOB_OK;
    int rc = check_msgs(c, m, n_steps);
    if (rc != LOB_OK) return rc;
    if ((rc = check_out(c, o)) != LOB_OK) return rc;
    KArgs a = base_args(c);
    fill_msgs(a, m);
    fill_out(a, o);
    a.actions_in = actions;
    a.t0 = c->t;
    a.n_steps = n_steps;
    rc = launch_env(c, a, (hipStream_t)stream);
    if (rc != LOB_OK) return rc;
    c->t += n_steps;
    return LOB_OK;
}

int lob_plan(lob_ctx *c, const lob_msgs *m, int32_t n_steps) {
    if (!c || n_steps <= 0) return LOB_EINVAL;
    int rc = check_msgs(c, m, 0);
    if (rc != LOB_OK) return rc;
    const int n = std::min(n_steps, m->n_steps - c->t);
    if (n <= 0) return LOB_ESTATE;
    return make_plan(c, m, c->t, n);
}

int lob_schedule_get(const lob_ctx *c, int32_t *out, int32_t max_classes) {
    if (!c || !out || max_classes < 0) return LOB_EINVAL;
    const int nc = (int)c->classes.size();
    for (int k = 0; k < nc && k < max_classes; ++k) {
        const CapClass &cl = c->classes[(size_t)k];
        int32_t *r = out + k * 5;
        r[0] = cl.capp; r[1] = cl.count; r[2] = cl.waves; r[3] = cl.mode; r[4] = cl.grid;
    }
    return nc;
}

int lob_schedule_set(lob_ctx *c, int32_t k, int32_t waves, int32_t mode, int32_t grid) {
    if (!c || k < 0 || k >= (int)c->classes.size()) return LOB_EINVAL;
    if (waves != 1 && waves != 2 && waves != 4) return LOB_EINVAL;
    if (mode != 0 && mode != 1) return LOB_EINVAL;
    if (grid < 0) return LOB_EINVAL;
    CapClass &cl = c->classes[(size_t)k];
    if ((size_t)lds_words_for(cl.capp, c->cfg.n_agents) * 4 * waves > 64 * 1024) return LOB_EUNSUPPORTED;
    cl.waves = waves;
    cl.mode = mode;
    cl.grid = grid;
    c->balance = 0; /* an explicit per-class schedule is kept by later plans */
    return LOB_OK;
}

int lob_schedule_balance(lob_ctx *c, int32_t permille) {
    if (!c || permille < 0 || permille > 1000) return LOB_EINVAL;
    c->balance = permille;
    if (permille == 0)
        for (CapClass &cl : c->classes) {
            cl.waves = default_waves(cl.capp, c->cfg.n_agents);
            cl.mode = 0;
            cl.grid = 0;
        }
    c->plan_off = nullptr; /* the next plan sizes the queues */
    c->plan_t0 = c->plan_steps = -1;
    return LOB_OK;
}

int lob_set_padded(lob_ctx *c, int32_t padded) {
    if (!c || (padded != 0 && padded != 1)) return LOB_EINVAL;
    if (!wait_launches(c)) return LOB_EHIP;
    return build_classes(c, padded != 0);
}

/* Time schedule candidates on the next n_steps of `m` from the current state (restored
 * after every run) and keep the fastest.  One class: every (waves, mode) of it.  Several
 * (concurrent) classes: the whole launch under the proportional work-queue schedule at
 * several LDS shares, and under per-class hardware dispatch.  Results do not depend on
 * the schedule.  Synchronous; `out` is scratch. */
int lob_autotune(lob_ctx *c, const lob_msgs *m, int32_t n_steps, const lob_out *o, void *stream) {
    if (!c || n_steps <= 0) return LOB_EINVAL;
    if (!c->reset_done || c->t + n_steps > c->cfg.episode_len) return LOB_ESTATE;
    int rc = check_msgs(c, m, n_steps);
    if (rc != LOB_OK) return rc;
    if ((rc = check_out(c, o)) != LOB_OK) return rc;
    if ((rc = make_plan(c, m, c->t, n_steps)) != LOB_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    const size_t N = (size_t)c->cfg.n_envs, A = (size_t)std::max(c->cfg.n_agents, 1);
    const size_t slots = N * 2 * (size_t)c->cfg.max_cap;
    /* save the state */
    struct Buf { void *dst; const void *src; size_t bytes; };
    std::vector<Buf> bufs;
    for (int f = 0; f < NF; ++f) bufs.push_back({nullptr, c->d_bk[f], slots * 4});
    bufs.push_back({nullptr, c->d_bk_n, N * 2 * 4});
    bufs.push_back({nullptr, c->d_env, N * ENVW * 8});
    bufs.push_back({nullptr, c->d_agent, N * A * AGW * 8});
    bufs.push_back({nullptr, c->d_ctr, N * LOB_N_COUNTERS * 8});
    bufs.push_back({nullptr, c->d_stats, N * STW * 8});
    for (Buf &b : bufs) {
        if (hipMalloc(&b.dst, b.bytes) != hipSuccess) {
            for (Buf &x : bufs) if (x.dst) (void)hipFree(x.dst);
            return LOB_ENOMEM;
        }
        if (!hip_ok(hipMemcpyAsync(b.dst, b.src, b.bytes, hipMemcpyDeviceToDevice, st))) rc = LOB_EHIP;
    }
    auto restore = [&]() {
        for (Buf &b : bufs)
            if (!hip_ok(hipMemcpyAsync(const_cast<void *>(b.src), b.dst, b.bytes, hipMemcpyDeviceToDevice, st)))
                rc = LOB_EHIP;
    };
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    KArgs a = base_args(c);
    fill_msgs(a, m);
    fill_out(a, o);
    a.t0 = c->t;
    a.n_steps = n_steps;
    if (c->classes.size() > 1) {
        int best_b = c->balance;
        float best = 1e30f;
        /* the rollout time falls and rises steeply around the best share (a few percent
         * per 40 permille), so the shares are 20 permille apart; each is run twice and
         * counts with its faster run */
        for (int b : {0, 800, 820, 840, 860, 880, 900, 920, 960}) {
            if (rc != LOB_OK) break;
            if ((rc = lob_schedule_balance(c, b)) != LOB_OK || (rc = make_plan(c, m, c->t, n_steps)) != LOB_OK)
                break;
            float ms = 1e30f;
            for (int rep = 0; rep < 2 && rc == LOB_OK; ++rep) {
                restore();
                (void)hipEventRecord(e0, st);
                rc = launch_env(c, a, st);
                (void)hipEventRecord(e1, st);
                (void)hipEventSynchronize(e1);
                float r = 0.f;
                (void)hipEventElapsedTime(&r, e0, e1);
                ms = std::min(ms, r);
            }
            if (rc == LOB_OK && ms < best) { best = ms; best_b = b; }
        }
        if (rc == LOB_OK) rc = lob_schedule_balance(c, best_b);
        if (rc == LOB_OK) rc = make_plan(c, m, c->t, n_steps);
    }
    for (size_t k = 0; k < c->classes.size() && c->classes.size() == 1 && rc == LOB_OK; ++k) {
        CapClass &cl = c->classes[k];
        const CapClass orig = cl;
        CapClass bestc = cl;
        float best = 1e30f;
        for (int mode = 0; mode < 2; ++mode) {
            for (int waves : {1, 2, 4}) {
                if ((size_t)lds_words_for(cl.capp, c->cfg.n_agents) * 4 * waves > 64 * 1024) continue;
                cl.waves = waves;
                cl.mode = mode;
                cl.grid = 0;
                float ms = 0.f;
                for (int rep = 0; rep < 2 && rc == LOB_OK; ++rep) {
                    restore();
                    (void)hipEventRecord(e0, st);
                    rc = launch_class(c, k, a, st);
                    (void)hipEventRecord(e1, st);
                    (void)hipEventSynchronize(e1);
                    (void)hipEventElapsedTime(&ms, e0, e1);
                }
                if (rc == LOB_OK && ms < best) { best = ms; bestc = cl; }
            }
        }
        cl = rc == LOB_OK ? bestc : orig;
    }
    restore();
    (void)hipStreamSynchronize(st);
    for (Buf &b : bufs) (void)hipFree(b.dst);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

int lob_observe(lob_ctx *c, float *obs, void *stream) {
    if (!c || (!obs && c->cfg.n_agents > 0)) return LOB_EINVAL;
    if (!c->reset_done) return LOB_ESTATE;
    if (c->cfg.n_agents == 0) return LOB_OK;
    KArgs a = base_args(c);
    a.obs = obs;
    for (const CapClass &cl : c->classes) {
        if (cl.count == 0) continue;
        a.capp = cl.capp;
        a.lds_words = lds_words_for(cl.capp, c->cfg.n_agents);
        a.env_list = c->d_env_list + cl.first;
        a.n_list = cl.count;
        const size_t lds = (size_t)a.lds_words * 4 * cl.waves;
        hipLaunchKernelGGL(k_observe, dim3((cl.count + cl.waves - 1) / cl.waves),
                           dim3(64 * cl.waves), lds, (hipStream_t)stream, a);
        if (hipGetLastError() != hipSuccess) return LOB_EHIP;
    }
    return LOB_OK;
}

int lob_export_books(lob_ctx *c, const lob_books *out, void *stream) {
    if (!c || !out || !out->price || !out->qty || !out->oid || !out->tid || !out->tsec || !out->tns || !out->n)
        return LOB_EINVAL;
    if (!c->reset_done) return LOB_ESTATE;
    ExportArgs a;
    std::memset(&a, 0, sizeof(a));
    a.n_envs = c->cfg.n_envs;
    a.n_agents = c->cfg.n_agents;
    a.max_cap = c->cfg.max_cap;
    int32_t *dst[NF] = {out->price, out->qty, out->oid, out->tid, out->tsec, out->tns};
    for (int f = 0; f < NF; ++f) { a.src[f] = c->d_bk[f]; a.dst[f] = dst[f]; }
    a.src_n = c->d_bk_n;
    a.dst_n = out->n;
    hipLaunchKernelGGL(k_export_books, dim3(1024), dim3(256), 0, (hipStream_t)stream, a);
    return hipGetLastError() == hipSuccess ? LOB_OK : LOB_EHIP;
}

int lob_export_state(lob_ctx *c, int64_t *env_state, int64_t *agent_state, int64_t *counters, void *stream) {
    if (!c) return LOB_EINVAL;
    if (!c->reset_done) return LOB_ESTATE;
    hipStream_t st = (hipStream_t)stream;
    const size_t N = (size_t)c->cfg.n_envs;
    ExportArgs a;
    std::memset(&a, 0, sizeof(a));
    a.n_envs = c->cfg.n_envs;
    a.n_agents = c->cfg.n_agents;
    a.agent_src = c->d_agent;
    a.agent_dst = agent_state;
    a.env_src = c->d_env;
    a.stats_src = c->d_stats;
    a.env_dst = env_state;
    if (env_state) {
        hipLaunchKernelGGL(k_export_env, dim3(64), dim3(256), 0, st, a);
        if (hipGetLastError() != hipSuccess) return LOB_EHIP;
    }
    if (counters && !hip_ok(hipMemcpyAsync(counters, c->d_ctr, N * LOB_N_COUNTERS * 8, hipMemcpyDeviceToDevice, st)))
        return LOB_EHIP;
    if (agent_state && c->cfg.n_agents > 0) {
        hipLaunchKernelGGL(k_export_agents, dim3(256), dim3(256), 0, st, a);
        if (hipGetLastError() != hipSuccess) return LOB_EHIP;
    }
    return LOB_OK;
}

int lob_import_state(lob_ctx *c, const lob_books *books, const int64_t *env_state, const int64_t *agent_state,
                     const int64_t *counters, int32_t step, void *stream) {
    if (!c || !books || !books->price || !books->qty || !books->oid || !books->tid || !books->tsec || !books->tns ||
        !books->n || !env_state || (c->cfg.n_agents > 0 && !agent_state))
        return LOB_EINVAL;
    if (step < 0 || step > c->cfg.episode_len) return LOB_EINVAL;
    ImportArgs a;
    std::memset(&a, 0, sizeof(a));
    a.n_envs = c->cfg.n_envs;
    a.n_agents = c->cfg.n_agents;
    a.max_cap = c->cfg.max_cap;
    a.step = step;
    a.caps = c->d_caps;
    const int32_t *src[NF] = {books->price, books->qty, books->oid, books->tid, books->tsec, books->tns};
    for (int f = 0; f < NF; ++f) { a.src[f] = src[f]; a.dst[f] = c->d_bk[f]; }
    a.src_n = books->n;
    a.env_src = env_state;
    a.agent_src = agent_state;
    a.ctr_src = counters;
    a.dst_n = c->d_bk_n;
    a.env_state = c->d_env;
    a.agent_state = c->d_agent;
    a.counters = c->d_ctr;
    a.stats = c->d_stats;
    const int waves = 4;
    hipLaunchKernelGGL(k_import, dim3((c->cfg.n_envs + waves - 1) / waves), dim3(64 * waves), 0, (hipStream_t)stream, a);
    if (hipGetLastError() != hipSuccess) return LOB_EHIP;
    c->t = step;
    c->reset_done = true;
    return LOB_OK;
}

} // extern "C"
