/*
 * Batched limit-order-book environment step: HIP kernels for gfx950 and the C-ABI.
 *
 * The step is the five-stage env step of JaxMARL-HFT (arXiv 2511.02136, Sec. 4):
 * action conversion with cancels (step 1), shuffle (step 2), concatenation with the
 * replayed messages (step 3), price-time-priority matching with trades recorded (step 4,
 * Sec. 2.1), and outcomes (step 5: fills, rewards by Eq. 2-4, observations).
 *
 * Design (MI355X-first):
 *   - one wavefront per environment; the book of both sides is LDS-resident as a
 *     structure of arrays, slot i in lane i%64 of row i/64 (see lob_device.h);
 *   - a book message is a handful of wave-wide LDS instructions: a ballot search for
 *     cancels, a wave prefix scan over the crossing quantities for matching (with a
 *     scalar fast path when the best order covers the incoming quantity), and a row
 *     shift for insertion / removal;
 *   - replay messages are staged 64 at a time with coalesced SoA loads, the next chunk
 *     prefetched while the current one is processed;
 *   - envs are grouped by capacity class (capacity rounded up to 64 slots) so each
 *     launch sizes LDS for its own class; the persistent form keeps books in LDS for all
 *     steps of a rollout and pulls envs from a device work queue, longest first.
 *
 * Floating point: rewards are evaluated in double in a fixed order with contraction
 * disabled and rounded once to float; observation features are exact integers rounded
 * to float.
 */
#include <hip/hip_runtime.h>

#include <algorithm>
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
constexpr int MAXLV = 8;          /* desired price levels per agent per step */
constexpr int MAXACT = MAXA * 8;  /* new agent orders per env-step */
constexpr int AGW = 8;            /* internal agent words: inv, cash, rem, ctr, step_bq, step_sq */
constexpr int STW = 4;            /* step statistics: buy vol, sell vol, trades, last price */

/* per-wave LDS layout (int32 words) after the book (12 * capp words) */
constexpr int X_ACT = 0;                    /* MAXACT x 8: ts, price, qty, oid, tid, tsec, tns, - */
constexpr int X_PERM = X_ACT + MAXACT * 8;  /* MAXACT: shuffled order */
constexpr int X_LV = X_PERM + MAXACT;       /* MAXLV x 4: side, price, desired qty, resting qty */
constexpr int X_SEEN = X_LV + MAXLV * 4;    /* MAXLV: older resting qty seen in the walk */
constexpr int X_AG = X_SEEN + MAXLV;        /* int64 MAXA x AGW */
constexpr int X_FL = X_AG + MAXA * AGW * 2; /* int64 MAXA x 4: fills of the step */
constexpr int X_OBK = X_FL + MAXA * 4 * 2;  /* int64 34: depth buckets, totals, own stats */
constexpr int N_OBK = 22 + 3 * MAXA;
constexpr int X_END = X_OBK + 34 * 2;
constexpr int EXTRA_WORDS = (X_END + 63) & ~63;
static_assert(N_OBK <= 34, "obs accumulator area");
static_assert((X_AG & 1) == 0 && (X_FL & 1) == 0 && (X_OBK & 1) == 0, "int64 alignment");

inline int lds_words_for(int capp) { return 2 * NF * capp + EXTRA_WORDS; }

struct KArgs {
    /* configuration */
    int32_t n_envs, n_agents, max_cap, episode_len;
    uint64_t seed;
    int32_t exec_task, exec_q0, mm_q, dir_q;
    float pen, lam, rho;
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
 * One environment run by one wavefront.
 * ---------------------------------------------------------------------------- */
struct Run {
    const KArgs &a;
    int32_t *L; /* this wave's LDS */
    int lane, capp, cap, e, A;
    /* book */
    int n0, n1, best0, best1;
    /* env state */
    int32_t last_bb, last_ba, last_tsec, last_tns, t;
    int64_t mid2_prev, p_init2, last_dmid2;
    int64_t ctr[NCTR];
    /* trade records */
    int64_t tr_base, tr_cap, tr_cur;
    /* per step */
    int64_t mid_sum, st_buy, st_sell, st_trades;
    int32_t mid_n, seq, st_last;

    __device__ Run(const KArgs &args, int32_t *lds, int env)
        : a(args), L(lds), lane(lane_id()), capp(args.capp), e(env), A(args.n_agents) {
        cap = a.caps[e];
    }

    /* ---- LDS views ---- */
    __device__ __forceinline__ int32_t &B(int s, int f, int i) { return L[(s * NF + f) * capp + i]; }
    __device__ __forceinline__ int32_t *X() { return L + 2 * NF * capp; }
    __device__ __forceinline__ int64_t *AG(int i) { return reinterpret_cast<int64_t *>(X() + X_AG) + i * AGW; }
    __device__ __forceinline__ int64_t *FL(int i) { return reinterpret_cast<int64_t *>(X() + X_FL) + i * 4; }
    __device__ __forceinline__ int64_t *OBK() { return reinterpret_cast<int64_t *>(X() + X_OBK); }
    __device__ __forceinline__ int32_t *LV(int k) { return X() + X_LV + k * 4; }

    __device__ __forceinline__ int nsz(int s) const { return s ? n1 : n0; }
    __device__ __forceinline__ void set_n(int s, int v) {
        if (s) n1 = v; else n0 = v;
    }
    __device__ __forceinline__ int best(int s) const { return s ? best1 : best0; }
    __device__ __forceinline__ void set_best(int s, int v) {
        if (s) best1 = v; else best0 = v;
    }
    __device__ __forceinline__ void refresh_best(int s) {
        int v = nsz(s) > 0 ? uni(B(s, FP, 0)) : 0;
        set_best(s, v);
    }

    /* ---- row shifts (wave-wide LDS copies) ---- */
    /* move slots [from, to) of side s to [from+1, to+1); to < capp */
    __device__ __forceinline__ void shift_up(int s, int from, int to) {
        if (to <= from) return;
        for (int r = to >> 6; r >= ((from + 1) >> 6); --r) {
            const int i = (r << 6) + lane;
            const bool mv = i > from && i <= to;
            int v[NF];
#pragma unroll
            for (int f = 0; f < NF; ++f) v[f] = mv ? B(s, f, max(i - 1, 0)) : 0;
            WAVE_SYNC();
            if (mv) {
#pragma unroll
                for (int f = 0; f < NF; ++f) B(s, f, i) = v[f];
            }
            WAVE_SYNC();
        }
    }
    /* remove k slots at [at, at+k) of a side holding n: [at+k, n) moves to [at, n-k) */
    __device__ __forceinline__ void shift_down(int s, int at, int k, int n) {
        const int newn = n - k;
        if (k <= 0 || at >= newn) return;
        for (int r = at >> 6; (r << 6) < newn; ++r) {
            const int i = (r << 6) + lane;
            const bool mv = i >= at && i < newn;
            int v[NF];
#pragma unroll
            for (int f = 0; f < NF; ++f) v[f] = mv ? B(s, f, min(i + k, capp - 1)) : 0;
            WAVE_SYNC();
            if (mv) {
#pragma unroll
                for (int f = 0; f < NF; ++f) B(s, f, i) = v[f];
            }
            WAVE_SYNC();
        }
    }
    __device__ __forceinline__ void put(int s, int i, int p, int q, int o, int tid, int ts, int tn) {
        if (lane == 0) {
            B(s, FP, i) = p; B(s, FQ, i) = q; B(s, FO, i) = o;
            B(s, FT, i) = tid; B(s, FS, i) = ts; B(s, FN, i) = tn;
        }
        WAVE_SYNC();
    }

    /* ---- fills (uniform accumulation in LDS by lane 0) ---- */
    __device__ __forceinline__ void add_fill(int tid, int buy, int64_t q, int64_t notional) {
        if (tid >= 1 && tid <= A) {
            if (lane == 0) {
                int64_t *f = FL(tid - 1) + (buy ? 0 : 2);
                f[0] += q;
                f[1] += notional;
            }
            WAVE_SYNC();
        }
    }

    /* ---- trade records ---- */
    __device__ __forceinline__ void write_trade(int64_t k, int price, int q, int agg_oid, int pas_oid,
                                                int agg_tid, int pas_tid, int side, int sq) {
        const int64_t rec = tr_cur + k;
        if (a.trades && rec < tr_cap) {
            int4 *p = reinterpret_cast<int4 *>(a.trades + (tr_base + rec) * LOB_TRADE_WORDS);
            p[0] = make_int4(price, q, agg_oid, pas_oid);
            p[1] = make_int4(agg_tid, pas_tid, side | (sq << 1), t);
        }
    }
    __device__ __forceinline__ void close_trades(int ntr, int64_t volume, int side, int last_price) {
        if (ntr <= 0) return;
        const int64_t end = tr_cur + ntr;
        const int64_t room = tr_cap > tr_cur ? tr_cap - tr_cur : 0;
        if (ntr > room) ctr[C_TRADE_OVERFLOW] += ntr - room;
        (void)end;
        tr_cur += ntr;
        ctr[C_TRADES] += ntr;
        st_trades += ntr;
        if (side == 0) st_buy += volume; else st_sell += volume;
        st_last = last_price;
    }

    /* ---- matching: an incoming order of side `side` against the opposite side while it
     * crosses (market orders cross at any price); trades at the resting price.  Returns
     * the unmatched remainder. ---- */
    __device__ int match(int side, int p, int q, bool market, int agg_oid, int agg_tid) {
        const int opp = 1 - side;
        const int no = nsz(opp);
        if (no == 0 || q <= 0) return q;
        const int bp = best(opp);
        if (!(market || (side == 0 ? bp <= p : bp >= p))) return q;
        const int bq = uni(B(opp, FQ, 0));
        if (bq >= q) {
            /* the best order alone covers the incoming quantity */
            const int poid = uni(B(opp, FO, 0));
            const int ptid = uni(B(opp, FT, 0));
            if (lane == 0) write_trade(0, bp, q, agg_oid, poid, agg_tid, ptid, side, seq);
            add_fill(agg_tid, side == 0, q, (int64_t)q * bp);
            add_fill(ptid, side != 0, q, (int64_t)q * bp);
            if (bq == q) {
                shift_down(opp, 0, 1, no);
                set_n(opp, no - 1);
                refresh_best(opp);
            } else {
                if (lane == 0) B(opp, FQ, 0) = bq - q;
                WAVE_SYNC();
            }
            close_trades(1, q, side, bp);
            return 0;
        }
        /* general case: prefix scan of the crossing quantities, row by row */
        int64_t carry = 0, my_notional = 0;
        int ntr = 0, nfull = 0, last_price = bp;
        const int rows = (no + 63) >> 6;
        for (int r = 0; r < rows; ++r) {
            const int i = (r << 6) + lane;
            const bool valid = i < no;
            const int pr = valid ? B(opp, FP, i) : 0;
            const int qt = valid ? B(opp, FQ, i) : 0;
            const bool cr = valid && (market || (side == 0 ? pr <= p : pr >= p));
            const int64_t x = cr ? (int64_t)qt : 0;
            const int64_t incl = wave_incl_scan64(x, lane) + carry;
            const int64_t excl = incl - x;
            const int take = (cr && excl < q) ? (int)min((int64_t)qt, (int64_t)q - excl) : 0;
            const bool has = take > 0;
            const uint64_t hm = ballot(has);
            int ptid = 0;
            if (has) {
                const int poid = B(opp, FO, i);
                ptid = B(opp, FT, i);
                write_trade(ntr + lane, pr, take, agg_oid, poid, agg_tid, ptid, side, seq);
                if (take < qt) B(opp, FQ, i) = qt - take;
                my_notional += (int64_t)take * pr;
            }
            WAVE_SYNC();
            /* resting orders of agents filled in this row (rare): accumulate uniformly */
            uint64_t pm = ballot(has && ptid >= 1 && ptid <= A);
            while (pm) {
                const int j = __builtin_ctzll(pm);
                pm &= pm - 1;
                const int tj = rdlane(ptid, j), kj = rdlane(take, j), pj = rdlane(pr, j);
                add_fill(tj, side != 0, kj, (int64_t)kj * pj);
            }
            nfull += __popcll(ballot(has && take == qt));
            const int c = __popcll(hm);
            if (c > 0) last_price = rdlane(pr, 63 - __builtin_clzll(hm));
            ntr += c;
            carry = rdlane64(incl, 63);
            if (carry >= q || ballot(cr) != ballot(valid)) break;
        }
        const int traded = (int)min((int64_t)q, carry);
        if (agg_tid >= 1 && agg_tid <= A) {
            const int64_t notional = uni64(wave_sum64(my_notional));
            add_fill(agg_tid, side == 0, traded, notional);
        }
        if (nfull > 0) {
            shift_down(opp, 0, nfull, no);
            set_n(opp, no - nfull);
            refresh_best(opp);
        }
        close_trades(ntr, traded, side, last_price);
        return q - traded;
    }

    /* ---- rest a limit remainder on its own side (after all orders at an equal or
     * better price); a full side evicts its worst order if the price is strictly
     * better than that order's, else the remainder is dropped. ---- */
    __device__ void rest(int side, int p, int q, int oid, int tid, int ts, int tn) {
        const int n = nsz(side);
        int pos = 0;
        const int rows = (n + 63) >> 6;
        for (int r = 0; r < rows; ++r) {
            const int i = (r << 6) + lane;
            const bool valid = i < n;
            const int pr = valid ? B(side, FP, i) : 0;
            const bool be = valid && (side == 0 ? pr >= p : pr <= p);
            const int c = __popcll(ballot(be));
            pos += c;
            if (c < 64) break;
        }
        if (n < cap) {
            shift_up(side, pos, n);
            put(side, pos, p, q, oid, tid, ts, tn);
            set_n(side, n + 1);
        } else {
            const int wp = uni(B(side, FP, n - 1));
            const bool better = side == 0 ? p > wp : p < wp;
            if (!better) {
                ctr[C_DROP] += 1;
                ctr[C_DROPPED_QTY] += q;
                return;
            }
            ctr[C_EVICT] += 1;
            ctr[C_EVICTED_QTY] += uni(B(side, FQ, n - 1));
            shift_up(side, pos, n - 1);
            put(side, pos, p, q, oid, tid, ts, tn);
        }
        if (pos == 0) set_best(side, p);
    }

    /* ---- cancels: the first order with this id on the message's side ---- */
    __device__ void cancel(bool partial, int side, int qty, int oid) {
        const int n = nsz(side);
        int found = -1;
        const int rows = (n + 63) >> 6;
        for (int r = 0; r < rows; ++r) {
            const int i = (r << 6) + lane;
            const uint64_t m = ballot(i < n && B(side, FO, i) == oid);
            if (m) {
                found = (r << 6) + __builtin_ctzll(m);
                break;
            }
        }
        if (found < 0) {
            ctr[C_MISS] += 1;
            return;
        }
        if (partial) {
            const int cq = uni(B(side, FQ, found));
            const int left = cq - min(qty, cq);
            if (left > 0) {
                if (lane == 0) B(side, FQ, found) = left;
                WAVE_SYNC();
                return;
            }
        }
        shift_down(side, found, 1, n);
        set_n(side, n - 1);
        if (found == 0) refresh_best(side);
    }

    /* ---- one message of the step sequence ---- */
    __device__ void process(int ts, int price, int qty, int oid, int tid, int tsec, int tns) {
        const int type = ts & 0xFF, side = (ts >> 8) & 1;
        ctr[C_MSGS] += 1;
        if (type == T_LIMIT || type == T_MARKET) {
            if (qty <= 0) {
                ctr[C_BAD] += 1;
            } else {
                const int q = match(side, price, qty, type == T_MARKET, oid, tid);
                if (type == T_MARKET) ctr[C_MARKET_UNFILLED] += q;
                else if (q > 0) rest(side, price, q, oid, tid, tsec, tns);
            }
        } else if (type == T_PCANCEL || type == T_DELETE) {
            if (type == T_PCANCEL && qty <= 0) ctr[C_BAD] += 1;
            else cancel(type == T_PCANCEL, side, qty, oid);
        } else {
            ctr[C_BAD] += 1;
        }
        last_tsec = tsec;
        last_tns = tns;
        if (n0 > 0 && n1 > 0) {
            mid_sum += (int64_t)best0 + best1;
            mid_n += 1;
        }
        seq += 1;
    }

    /* ---- desired levels of one agent (LDS, written by lane 0) ---- */
    __device__ __forceinline__ void add_level(int &nlv, int side, int price, int qty) {
        int k = 0;
        for (; k < nlv; ++k)
            if (uni(LV(k)[0]) == side && uni(LV(k)[1]) == price) break;
        if (k < nlv) {
            if (lane == 0) LV(k)[2] += qty;
        } else if (nlv < MAXLV) {
            if (lane == 0) {
                LV(k)[0] = side; LV(k)[1] = price; LV(k)[2] = qty; LV(k)[3] = 0;
            }
            nlv += 1;
        }
        WAVE_SYNC();
    }
    __device__ __forceinline__ int find_level(int nlv, int side, int price) {
        for (int k = 0; k < nlv; ++k)
            if (uni(LV(k)[0]) == side && uni(LV(k)[1]) == price) return k;
        return -1;
    }
    /* first index >= i0 on side s holding an order of trader tid, or -1 */
    __device__ __forceinline__ int next_own(int s, int i0, int tid) {
        const int n = nsz(s);
        for (int r = i0 >> 6; (r << 6) < n; ++r) {
            const int i = (r << 6) + lane;
            const uint64_t m = ballot(i >= i0 && i < n && B(s, FT, i) == tid);
            if (m) return (r << 6) + __builtin_ctzll(m);
        }
        return -1;
    }

    /* Sec. 4 step 1 for agent i: decode its action into desired levels (Sec. 4.1),
     * then cancel / top up its resting orders against them; new orders are appended to
     * the action block. */
    __device__ void agent_actions(int i, int act, int bb0, int ba0, int &nact) {
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
                        else add_level(nlv, 1, pp[k], (int)q);
                    }
                }
            }
        } else if (kind == LOB_AGENT_MM) {
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
                for (int o = 0; o < 4; ++o) add_level(nlv, 0, min(bb0 - o, ba0 - 1), q);
                for (int o = 0; o < 4; ++o) add_level(nlv, 1, max(ba0 + o, bb0 + 1), q);
            } else {
                if (hb) add_level(nlv, 0, min(bb0 - ob, ba0 - 1), q);
                if (ha) add_level(nlv, 1, max(ba0 + oa, bb0 + 1), q);
            }
        } else {
            /* directional: take the opposite touch with a fixed quantity */
            if (act == 1) add_level(nlv, 0, ba0, a.dir_q);
            if (act == 2) add_level(nlv, 1, bb0, a.dir_q);
        }

        /* resting quantity of this agent at each desired level (step start) */
        for (int s = 0; s < 2; ++s) {
            int i0 = 0;
            for (;;) {
                const int j = next_own(s, i0, tid);
                if (j < 0) break;
                const int k = find_level(nlv, s, uni(B(s, FP, j)));
                if (k >= 0) {
                    if (lane == 0) LV(k)[3] += B(s, FQ, j);
                    WAVE_SYNC();
                }
                i0 = j + 1;
            }
        }
        if (lane < MAXLV) X()[X_SEEN + lane] = 0;
        WAVE_SYNC();
        /* walk the agent's resting orders in book order (bids, then asks): delete those at
         * levels it no longer wants; at a kept level take any excess from the newest */
        for (int s = 0; s < 2; ++s) {
            int i0 = 0;
            for (;;) {
                const int j = next_own(s, i0, tid);
                if (j < 0) break;
                const int pr = uni(B(s, FP, j)), qt = uni(B(s, FQ, j)), oid = uni(B(s, FO, j));
                const int k = find_level(nlv, s, pr);
                const int D = k >= 0 ? uni(LV(k)[2]) : 0;
                if (D == 0) {
                    process(T_DELETE | (s << 8), pr, qt, oid, tid, last_tsec, last_tns);
                    i0 = j;
                    continue;
                }
                const int R = uni(LV(k)[3]);
                const int older = uni(X()[X_SEEN + k]);
                if (lane == 0) X()[X_SEEN + k] = older + qt;
                WAVE_SYNC();
                if (R > D) {
                    const int need = R - D;
                    const int newer = R - older - qt;
                    const int x = min(max(need - newer, 0), qt);
                    if (x > 0) {
                        process(T_PCANCEL | (s << 8), pr, x, oid, tid, last_tsec, last_tns);
                        i0 = (x == qt) ? j : j + 1;
                        continue;
                    }
                }
                i0 = j + 1;
            }
        }
        /* new orders: the difference to the desired quantity, then any market order */
        auto append = [&](int type, int side, int price, int qty) {
            int64_t *g = AG(i);
            const int64_t c = uni64(g[3]);
            const int oid = (int)((1u << 30) | ((uint32_t)i << 26) | (uint32_t)(c & ((1 << 26) - 1)));
            if (lane == 0) {
                int32_t *m = X() + X_ACT + nact * 8;
                m[0] = type | (side << 8); m[1] = price; m[2] = qty; m[3] = oid;
                m[4] = tid; m[5] = last_tsec; m[6] = last_tns;
                g[3] = c + 1;
            }
            WAVE_SYNC();
            nact += 1;
        };
        for (int k = 0; k < nlv; ++k) {
            const int D = uni(LV(k)[2]), R = uni(LV(k)[3]);
            if (D > R) append(T_LIMIT, uni(LV(k)[0]), uni(LV(k)[1]), D - R);
        }
        if (mkt > 0) append(T_MARKET, 1, 0, (int)mkt);
    }

    /* ---- observation features from the book (LDS accumulators) ---- */
    __device__ void book_obs() {
        int64_t *O = OBK();
        if (lane < 34) O[lane] = 0;
        WAVE_SYNC();
        const int bb = last_bb, ba = last_ba;
        for (int s = 0; s < 2; ++s) {
            const int n = nsz(s);
            int64_t tot = 0;
            for (int r = 0; (r << 6) < n; ++r) {
                const int i = (r << 6) + lane;
                if (i < n) {
                    const int pr = B(s, FP, i), qt = B(s, FQ, i), td = B(s, FT, i);
                    const int64_t d = s == 0 ? (int64_t)bb - pr : (int64_t)pr - ba;
                    if (d >= 0 && d <= 9)
                        atomicAdd(reinterpret_cast<unsigned long long *>(O + s * 10 + d), (unsigned long long)qt);
                    if (td >= 1 && td <= A) {
                        atomicAdd(reinterpret_cast<unsigned long long *>(O + 22 + 3 * (td - 1) + s),
                                  (unsigned long long)qt);
                        atomicAdd(reinterpret_cast<unsigned long long *>(O + 22 + 3 * (td - 1) + 2), 1ull);
                    }
                    tot += qt;
                }
            }
            tot = wave_sum64(tot);
            WAVE_SYNC();
            if (lane == 0) O[20 + s] = tot;
            WAVE_SYNC();
        }
    }
    /* write the 40 features of every agent for output step slot s_idx */
    __device__ void write_obs(float *base /* [A][n_envs][40] */) {
        book_obs();
        const int64_t *O = OBK();
        const int64_t mid2 = (int64_t)last_bb + last_ba;
        for (int i = 0; i < A; ++i) {
            const int kind = (a.kinds >> (4 * i)) & 15;
            const int64_t *g = AG(i);
            int64_t v = 0;
            const int f = lane;
            if (f >= 3 && f <= 24) v = O[f - 3];
            else if (f >= 35 && f <= 37) v = O[22 + 3 * i + (f - 35)];
            else if (f == 0) v = (int64_t)last_ba - last_bb;
            else if (f == 1) v = last_dmid2;
            else if (f == 2) v = mid2 - p_init2;
            else if (f == 25) v = n0;
            else if (f == 26) v = n1;
            else if (f == 27) v = st_buy;
            else if (f == 28) v = st_sell;
            else if (f == 29) v = st_trades;
            else if (f == 30) v = st_trades > 0 ? 2 * (int64_t)st_last - mid2 : 0;
            else if (f == 31) v = g[0];
            else if (f == 32) v = g[1];
            else if (f == 33) v = kind == LOB_AGENT_EXEC ? g[2] : 0;
            else if (f == 34) v = (int64_t)a.episode_len - t;
            else if (f == 38) v = g[4];
            else if (f == 39) v = g[5];
            if (f < LOB_OBS_DIM) base[((int64_t)i * a.n_envs + e) * LOB_OBS_DIM + f] = (float)v;
        }
    }

    /* ---- load / store of the env ---- */
    __device__ void load() {
        const int64_t gb = (int64_t)e * 2;
        n0 = min(uni(a.bk_n[gb]), cap);
        n1 = min(uni(a.bk_n[gb + 1]), cap);
        for (int s = 0; s < 2; ++s) {
            const int n = nsz(s);
            const int64_t off = (gb + s) * a.max_cap;
            for (int i = lane; i < n; i += WAVE) {
#pragma unroll
                for (int f = 0; f < NF; ++f) B(s, f, i) = a.bk[f][off + i];
            }
        }
        WAVE_SYNC();
        refresh_best(0);
        refresh_best(1);
        const int64_t *es = a.env_state + (int64_t)e * LOB_ENV_STATE_WORDS;
        last_bb = (int32_t)uni64(es[0]);
        last_ba = (int32_t)uni64(es[1]);
        mid2_prev = uni64(es[2]);
        p_init2 = uni64(es[3]);
        last_tsec = (int32_t)uni64(es[4]);
        last_tns = (int32_t)uni64(es[5]);
        t = (int32_t)uni64(es[6]);
        last_dmid2 = uni64(es[7]);
#pragma unroll
        for (int k = 0; k < NCTR; ++k) ctr[k] = uni64(a.counters[(int64_t)e * LOB_N_COUNTERS + k]);
        const int64_t *st = a.stats + (int64_t)e * STW;
        st_buy = uni64(st[0]);
        st_sell = uni64(st[1]);
        st_trades = uni64(st[2]);
        st_last = (int32_t)uni64(st[3]);
        const int64_t *ag = a.agent_state + (int64_t)e * A * AGW;
        if (lane < A * AGW) AG(0)[lane] = ag[lane];
        tr_base = a.trade_off ? a.trade_off[e] : 0;
        tr_cap = a.trades ? a.trade_off[e + 1] - tr_base : 0;
        tr_cur = a.trade_cursor ? uni64(a.trade_cursor[e]) : 0;
        WAVE_SYNC();
    }
    __device__ void store() {
        WAVE_SYNC();
        const int64_t gb = (int64_t)e * 2;
        for (int s = 0; s < 2; ++s) {
            const int n = nsz(s);
            const int64_t off = (gb + s) * a.max_cap;
            for (int i = lane; i < n; i += WAVE) {
#pragma unroll
                for (int f = 0; f < NF; ++f) a.bk[f][off + i] = B(s, f, i);
            }
        }
        if (lane == 0) {
            a.bk_n[gb] = n0;
            a.bk_n[gb + 1] = n1;
        }
        int64_t *es = a.env_state + (int64_t)e * LOB_ENV_STATE_WORDS;
        int64_t v = 0;
        switch (lane) {
        case 0: v = last_bb; break;
        case 1: v = last_ba; break;
        case 2: v = mid2_prev; break;
        case 3: v = p_init2; break;
        case 4: v = last_tsec; break;
        case 5: v = last_tns; break;
        case 6: v = t; break;
        case 7: v = last_dmid2; break;
        default: break;
        }
        if (lane < LOB_ENV_STATE_WORDS) es[lane] = v;
        int64_t c = 0;
#pragma unroll
        for (int k = 0; k < NCTR; ++k)
            if (lane == k) c = ctr[k];
        if (lane < NCTR) a.counters[(int64_t)e * LOB_N_COUNTERS + lane] = c;
        int64_t sv = lane == 0 ? st_buy : lane == 1 ? st_sell : lane == 2 ? st_trades : (int64_t)st_last;
        if (lane < STW) a.stats[(int64_t)e * STW + lane] = sv;
        int64_t *ag = a.agent_state + (int64_t)e * A * AGW;
        if (lane < A * AGW) ag[lane] = AG(0)[lane];
        if (a.trade_cursor && lane == 0) a.trade_cursor[e] = tr_cur;
    }

    /* ---- one env-step (Sec. 4 steps 1-5) writing output slot s_idx ---- */
    __device__ void step(int s_idx) {
        const int N = a.n_envs;
        mid_sum = 0; mid_n = 0; seq = 0;
        st_buy = 0; st_sell = 0; st_trades = 0; st_last = 0;
        if (lane < A * 4) FL(0)[lane] = 0;
        WAVE_SYNC();
        /* reference prices at step start; an empty side keeps its last known best */
        const int bb0 = n0 > 0 ? best0 : last_bb;
        const int ba0 = n1 > 0 ? best1 : last_ba;

        /* step 1: action conversion, agents in index order; cancels processed at once */
        int nact = 0;
        for (int i = 0; i < A; ++i) {
            const int kind = (a.kinds >> (4 * i)) & 15;
            const int nacts = kind == LOB_AGENT_DIR ? 3 : 9;
            int act;
            if (a.actions_in) {
                act = uni(a.actions_in[((int64_t)s_idx * A + i) * N + e]);
            } else {
                const uint32_t u = (uint32_t)(hash4(a.seed, DOM_ACTION, (uint64_t)e, (uint64_t)t, (uint64_t)i) >> 32);
                act = (int)(((uint64_t)u * (uint64_t)nacts) >> 32);
            }
            if (a.actions_out && lane == 0) a.actions_out[((int64_t)s_idx * A + i) * N + e] = act;
            if (act < 0 || act >= nacts) act = 0;
            agent_actions(i, act, bb0, ba0, nact);
        }

        /* step 2: shuffle the new orders by (32-bit counter hash, position) */
        if (nact > 0) {
            const uint32_t key = (uint32_t)(hash4(a.seed, DOM_SHUFFLE, (uint64_t)e, (uint64_t)t, (uint64_t)lane) >> 32);
            int rank = 0;
            for (int j = 0; j < nact; ++j) {
                const uint32_t kj = (uint32_t)rdlane((int)key, j);
                rank += (kj < key || (kj == key && j < lane)) ? 1 : 0;
            }
            if (lane < nact) X()[X_PERM + rank] = lane;
            WAVE_SYNC();
            /* step 3 (first part): the shuffled action block follows the cancels */
            for (int p = 0; p < nact; ++p) {
                const int k = uni(X()[X_PERM + p]);
                const int32_t *m = X() + X_ACT + k * 8;
                process(uni(m[0]), uni(m[1]), uni(m[2]), uni(m[3]), uni(m[4]), uni(m[5]), uni(m[6]));
            }
        }

        /* step 3 (second part) + step 4: the replayed messages, staged 64 at a time */
        const int64_t *row = a.m_off + (int64_t)e * (a.m_steps + 1);
        const int64_t lo = uni64(row[t]), hi = uni64(row[t + 1]);
        int64_t base = lo;
        int c0 = 0, c1 = 0, c2 = 0, c3 = 0, c4 = 0, c5 = 0, c6 = 0;
        if (base < hi) {
            const int64_t idx = base + lane;
            if (idx < hi) {
                c0 = a.m_ts[idx]; c1 = a.m_price[idx]; c2 = a.m_qty[idx]; c3 = a.m_oid[idx];
                c4 = a.m_tid[idx]; c5 = a.m_tsec[idx]; c6 = a.m_tns[idx];
            }
        }
        while (base < hi) {
            const int64_t nb = base + WAVE;
            int d0 = 0, d1 = 0, d2 = 0, d3 = 0, d4 = 0, d5 = 0, d6 = 0;
            const int64_t nidx = nb + lane;
            if (nidx < hi) {
                d0 = a.m_ts[nidx]; d1 = a.m_price[nidx]; d2 = a.m_qty[nidx]; d3 = a.m_oid[nidx];
                d4 = a.m_tid[nidx]; d5 = a.m_tsec[nidx]; d6 = a.m_tns[nidx];
            }
            const int cnt = (int)min((int64_t)WAVE, hi - base);
            for (int j = 0; j < cnt; ++j)
                process(rdlane(c0, j), rdlane(c1, j), rdlane(c2, j), rdlane(c3, j), rdlane(c4, j),
                        rdlane(c5, j), rdlane(c6, j));
            c0 = d0; c1 = d1; c2 = d2; c3 = d3; c4 = d4; c5 = d5; c6 = d6;
            base = nb;
        }

        /* step 5: outcomes */
        const int bb1 = n0 > 0 ? best0 : last_bb;
        const int ba1 = n1 > 0 ? best1 : last_ba;
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
            const int64_t rem = uni64(g[2]) - (kind == LOB_AGENT_EXEC ? sq : 0);
            const double psi_b = mbar * (double)bq - (double)bn;
            const double psi_s = (double)sn - mbar * (double)sq;
            double r;
            if (kind == LOB_AGENT_MM) {
                /* Eq. 3 with the quadratic inventory penalty */
                const double psi_inv = (double)inv * (mt - mprev);
                const double pos = psi_inv > 0.0 ? psi_inv : 0.0;
                r = psi_b + psi_s + psi_inv - (1.0 - (double)a.lam) * pos - (double)a.rho * ((double)inv * (double)inv);
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
        WAVE_SYNC();
        last_dmid2 = mid2_end - mid2_prev;
        last_bb = bb1;
        last_ba = ba1;
        mid2_prev = mid2_end;
        t += 1;
        if (lane == 0) {
            a.n_trades[(int64_t)s_idx * N + e] = (int32_t)st_trades;
            a.done[(int64_t)s_idx * N + e] = last ? 1 : 0;
        }
        if (a.obs) write_obs(a.obs + (int64_t)s_idx * A * N * LOB_OBS_DIM);
    }
};

/* ------------------------------------------------------------------------------
 * Kernels
 * ---------------------------------------------------------------------------- */
__global__ void __launch_bounds__(256) k_env(KArgs a) {
    extern __shared__ int32_t smem[];
    const int wave = (int)(threadIdx.x >> 6), waves = (int)(blockDim.x >> 6);
    int32_t *L = smem + (int64_t)wave * a.lds_words;
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
    const int wave = (int)(threadIdx.x >> 6), waves = (int)(blockDim.x >> 6);
    const int slot = (int)blockIdx.x * waves + wave;
    if (slot >= a.n_list) return;
    int32_t *L = smem + (int64_t)wave * a.lds_words;
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
    if (lane < LOB_ENV_STATE_WORDS) a.env_state[(int64_t)e * LOB_ENV_STATE_WORDS + lane] = v;
    if (lane < LOB_N_COUNTERS) a.counters[(int64_t)e * LOB_N_COUNTERS + lane] = 0;
    if (lane < STW) a.stats[(int64_t)e * STW + lane] = 0;
    if (lane < a.n_agents * AGW) {
        const int i = lane / AGW, w = lane % AGW;
        const int kind = (a.kinds >> (4 * i)) & 15;
        a.agent_state[(int64_t)e * a.n_agents * AGW + lane] = (w == 2 && kind == LOB_AGENT_EXEC) ? (int64_t)a.exec_task : 0;
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
    int capp;      /* capacity rounded up to a multiple of 64 */
    int first;     /* offset into the env list */
    int count;     /* envs in the class */
    int waves;     /* waves per workgroup (envs per workgroup) */
};

struct lob_ctx {
    lob_config cfg;
    std::vector<int32_t> caps, kinds;
    int32_t kinds_packed = 0;
    int32_t *d_caps = nullptr;
    int32_t *d_bk[NF] = {};
    int32_t *d_bk_n = nullptr;
    int64_t *d_env = nullptr, *d_agent = nullptr, *d_ctr = nullptr, *d_stats = nullptr;
    int32_t *d_env_list = nullptr;  /* envs grouped by class */
    int32_t *d_work = nullptr;      /* work-queue counters, one per class */
    std::vector<CapClass> classes;
    int device = 0;
    int n_cu = 256;
    int t = 0;
    bool reset_done = false;
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

/* launch the env kernel for every capacity class */
int launch_env(lob_ctx *c, KArgs a, bool persistent, hipStream_t st) {
    for (size_t k = 0; k < c->classes.size(); ++k) {
        const CapClass &cl = c->classes[k];
        if (cl.count == 0) continue;
        a.capp = cl.capp;
        a.lds_words = lds_words_for(cl.capp);
        a.env_list = c->d_env_list + cl.first;
        a.n_list = cl.count;
        const int waves = cl.waves;
        const size_t lds = (size_t)a.lds_words * 4 * waves;
        int grid;
        if (persistent) {
            a.work_ctr = c->d_work + k;
            hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, c->d_work + k, 1, 0);
            int per_cu = (int)(160 * 1024 / lds);
            if (per_cu < 1) per_cu = 1;
            grid = std::min((cl.count + waves - 1) / waves, c->n_cu * per_cu);
        } else {
            a.work_ctr = nullptr;
            grid = (cl.count + waves - 1) / waves;
        }
        hipLaunchKernelGGL(k_env, dim3(grid), dim3(64 * waves), lds, st, a);
        if (hipGetLastError() != hipSuccess) return LOB_EHIP;
    }
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
        if (k < 0 || k > 2) { delete c; return LOB_EINVAL; }
        c->kinds.push_back(k);
        c->kinds_packed |= k << (4 * i);
    }
    c->cfg.cap = nullptr;
    c->cfg.agent_kind = nullptr;
    if (!hip_ok(hipGetDevice(&c->device))) { delete c; return LOB_EHIP; }
    hipDeviceProp_t prop;
    if (hip_ok(hipGetDeviceProperties(&prop, c->device))) c->n_cu = prop.multiProcessorCount;

    const int64_t N = cfg->n_envs, A = cfg->n_agents;
    const size_t slots = (size_t)N * 2 * cfg->max_cap;
    int rc = LOB_OK;
    rc |= dalloc(&c->d_caps, (size_t)N);
    for (int f = 0; f < NF; ++f) rc |= dalloc(&c->d_bk[f], slots);
    rc |= dalloc(&c->d_bk_n, (size_t)N * 2);
    rc |= dalloc(&c->d_env, (size_t)N * LOB_ENV_STATE_WORDS);
    rc |= dalloc(&c->d_agent, (size_t)(N * std::max<int64_t>(A, 1) * AGW));
    rc |= dalloc(&c->d_ctr, (size_t)N * LOB_N_COUNTERS);
    rc |= dalloc(&c->d_stats, (size_t)N * STW);
    rc |= dalloc(&c->d_env_list, (size_t)N);
    rc |= dalloc(&c->d_work, 64);
    if (rc != LOB_OK) { free_ctx(c); return LOB_ENOMEM; }

    /* capacity classes: capacity rounded up to 64 slots; envs of a class listed in
     * index order (the persistent launch reorders by work, see lob_rollout) */
    std::vector<int32_t> list;
    std::vector<int> cps;
    for (int32_t v : c->caps) cps.push_back((v + 63) & ~63);
    std::vector<int> uniq(cps);
    std::sort(uniq.begin(), uniq.end());
    uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
    for (int capp : uniq) {
        CapClass cl{capp, (int)list.size(), 0, 1};
        for (int e = 0; e < (int)N; ++e)
            if (cps[(size_t)e] == capp) { list.push_back(e); cl.count++; }
        /* several waves per workgroup when books are small */
        const size_t per_wave = (size_t)lds_words_for(capp) * 4;
        cl.waves = per_wave * 4 <= 64 * 1024 ? 4 : per_wave * 2 <= 64 * 1024 ? 2 : 1;
        c->classes.push_back(cl);
    }
    if (!hip_ok(hipMemcpy(c->d_caps, c->caps.data(), (size_t)N * 4, hipMemcpyHostToDevice)) ||
        !hip_ok(hipMemcpy(c->d_env_list, list.data(), (size_t)N * 4, hipMemcpyHostToDevice))) {
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
    rc = launch_env(c, a, false, (hipStream_t)stream);
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
    rc = launch_env(c, a, true, (hipStream_t)stream);
    if (rc != LOB_OK) return rc;
    c->t += n_steps;
    return LOB_OK;
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
        a.lds_words = lds_words_for(cl.capp);
        a.env_list = c->d_env_list + cl.first;
        a.n_list = cl.count;
        const size_t lds = (size_t)a.lds_words * 4 * cl.waves;
        hipLaunchKernelGGL(k_observe, dim3((cl.count + cl.waves - 1) / cl.waves), dim3(64 * cl.waves), lds,
                           (hipStream_t)stream, a);
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
    if (env_state && !hip_ok(hipMemcpyAsync(env_state, c->d_env, N * LOB_ENV_STATE_WORDS * 8, hipMemcpyDeviceToDevice, st)))
        return LOB_EHIP;
    if (counters && !hip_ok(hipMemcpyAsync(counters, c->d_ctr, N * LOB_N_COUNTERS * 8, hipMemcpyDeviceToDevice, st)))
        return LOB_EHIP;
    if (agent_state && c->cfg.n_agents > 0) {
        ExportArgs a;
        std::memset(&a, 0, sizeof(a));
        a.n_envs = c->cfg.n_envs;
        a.n_agents = c->cfg.n_agents;
        a.agent_src = c->d_agent;
        a.agent_dst = agent_state;
        hipLaunchKernelGGL(k_export_agents, dim3(256), dim3(256), 0, st, a);
        if (hipGetLastError() != hipSuccess) return LOB_EHIP;
    }
    return LOB_OK;
}

} // extern "C"
