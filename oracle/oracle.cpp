/*
 * CPU oracle for the batched limit-order-book environment step.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path.  It shares no code with
 * the HIP library.
 *
 * Deliberately plain and sequential.  Each side of a book is a std::map from price
 * to a FIFO deque of resting orders, so price priority is the map order and time
 * priority is the deque order (Sec. 2.1: a continuous double auction matches by price,
 * then by time).  Cancels search the side in priority order.  The environment step
 * follows the five stages listed in Sec. 4 one after another, for one env at a time.
 *
 * Readings of points the paper leaves open are marked "Reading:" below; each one is
 * listed in the design notes of the repository.
 */
#include "oracle.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <thread>
#include <vector>

namespace {

enum { LIMIT = 1, PARTIAL_CANCEL = 2, DELETE = 3, MARKET = 4, EXECUTE = 5, IGNORED = 6 };
enum { BUY = 0, SELL = 1 };
enum { AG_EXEC = 0, AG_MM = 1, AG_DIR = 2, AG_MM_BUYSELL = 3, AG_MM_SPREADSKEW = 4, AG_MM_AVST = 5,
       AG_EXEC_TWAP = 6, AG_MM_AS = 7 };
bool is_exec(int kind) { return kind == AG_EXEC || kind == AG_EXEC_TWAP; }
/* market makers rewarded by Eq. 3 (Spooner) */
bool is_spooner(int kind) { return kind == AG_MM || kind == AG_MM_SPREADSKEW || kind == AG_MM_AVST || kind == AG_MM_AS; }
/* per-env counters */
enum { C_MSGS, C_TRADES, C_MISS, C_EVICT, C_EVICTED_QTY, C_DROP, C_DROPPED_QTY,
       C_MARKET_UNFILLED, C_BAD, C_TRADE_OVERFLOW, C_IGNORED, N_COUNTERS };
constexpr int OBS_DIM = 40;
constexpr int TRADE_WORDS = 8;
constexpr int ENV_WORDS = 12;   /* exported env state words per env */
constexpr int AGENT_WORDS = 6; /* exported agent state words per agent */

/* ------------------------------------------------------------------------------
 * Counter hash: SplitMix64's output function (Steele, Lea, Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014), chained over the key words.
 * ---------------------------------------------------------------------------- */
uint64_t splitmix64_mix(uint64_t z) {
    z += 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
uint64_t chain_hash(uint64_t seed, uint64_t dom, uint64_t a, uint64_t b, uint64_t c) {
    return splitmix64_mix(splitmix64_mix(splitmix64_mix(splitmix64_mix(seed ^ dom) ^ a) ^ b) ^ c);
}
constexpr uint64_t DOM_SHUFFLE = 0x5348554646ULL; /* "SHUFF" */
constexpr uint64_t DOM_ACTION = 0x414354ULL;      /* "ACT" */

struct Order {
    int32_t price, qty, oid, tid, tsec, tns;
};

struct Msg {
    int32_t type, side, price, qty, oid, tid, tsec, tns;
};

/* One side of the book.  Key: -price for bids, +price for asks, so begin() is the best
 * level; within a level the deque front is the oldest order. */
struct Side {
    bool bid;
    std::map<int64_t, std::deque<Order>> levels;
    int32_t count = 0;

    explicit Side(bool is_bid) : bid(is_bid) {}
    int64_t key(int32_t price) const { return bid ? -(int64_t)price : (int64_t)price; }
    bool empty() const { return count == 0; }
    Order &best() { return levels.begin()->second.front(); }
    void pop_best() {
        auto it = levels.begin();
        it->second.pop_front();
        if (it->second.empty()) levels.erase(it);
        --count;
    }
    Order &worst() { return std::prev(levels.end())->second.back(); }
    void pop_worst() {
        auto it = std::prev(levels.end());
        it->second.pop_back();
        if (it->second.empty()) levels.erase(it);
        --count;
    }
    /* Time priority: a new order joins the back of its price level. */
    void insert(const Order &o) {
        levels[key(o.price)].push_back(o);
        ++count;
    }
    /* The first order with this id in priority order, or nullptr. */
    Order *find(int32_t oid, int64_t *level_key, size_t *pos) {
        for (auto &lv : levels) {
            for (size_t j = 0; j < lv.second.size(); ++j) {
                if (lv.second[j].oid == oid) {
                    *level_key = lv.first;
                    *pos = j;
                    return &lv.second[j];
                }
            }
        }
        return nullptr;
    }
    void erase(int64_t level_key, size_t pos) {
        auto it = levels.find(level_key);
        it->second.erase(it->second.begin() + (std::ptrdiff_t)pos);
        if (it->second.empty()) levels.erase(it);
        --count;
    }
    /* All orders in priority order. */
    std::vector<Order> list() const {
        std::vector<Order> v;
        for (const auto &lv : levels)
            for (const auto &o : lv.second) v.push_back(o);
        return v;
    }
    void load(const std::vector<Order> &v) {
        levels.clear();
        count = 0;
        for (const auto &o : v) insert(o);
    }
};

/* Sink for trade records of one message sequence. */
struct TradeSink {
    int32_t *buf = nullptr;   /* may be null: records are then not written */
    int64_t cap = 0;          /* records that fit */
    int64_t written = 0;      /* records produced so far (written or not) */
    int64_t *counters = nullptr;
    std::vector<int32_t> *step = nullptr; /* every record of the current step */
};

struct Book {
    int32_t cap;
    Side bids{true}, asks{false};
    explicit Book(int32_t c) : cap(c) {}
    Side &side(int s) { return s == BUY ? bids : asks; }
    bool both() const { return bids.count > 0 && asks.count > 0; }
};

/* Trade at the resting (passive) order's price.  Reading: the paper defers matching to
 * the JAX-LOB simulator; textbook price-time priority trades at the passive price. */
void emit_record(TradeSink &ts, const int32_t (&rec)[TRADE_WORDS]) {
    if (ts.written < ts.cap && ts.buf) {
        std::memcpy(ts.buf + ts.written * TRADE_WORDS, rec, sizeof(rec));
    } else {
        ts.counters[C_TRADE_OVERFLOW] += 1;
    }
    if (ts.step) ts.step->insert(ts.step->end(), rec, rec + TRADE_WORDS);
    ts.written += 1;
    ts.counters[C_TRADES] += 1;
}
/* the incoming message m is the aggressor */
void emit_trade(TradeSink &ts, int32_t price, int32_t x, const Msg &m, const Order &p, int32_t seq,
                int32_t t) {
    const int32_t rec[TRADE_WORDS] = {price, x, m.oid, p.oid, m.tid, p.tid, m.side | (seq << 1), t};
    emit_record(ts, rec);
}

/* Match an incoming order against the opposite side while it crosses (a market order
 * crosses at any price).  Returns the unmatched remainder. */
int32_t match(Book &bk, const Msg &m, bool market, TradeSink &ts, int32_t seq, int32_t t) {
    Side &opp = bk.side(1 - m.side);
    int32_t q = m.qty;
    while (q > 0 && !opp.empty()) {
        Order &b = opp.best();
        bool crosses = market || (m.side == BUY ? b.price <= m.price : b.price >= m.price);
        if (!crosses) break;
        int32_t x = std::min(q, b.qty);
        emit_trade(ts, b.price, x, m, b, seq, t);
        b.qty -= x;
        q -= x;
        if (b.qty == 0) opp.pop_best();
    }
    return q;
}

/* Process one message (Sec. 4 step 4).  Message types (Reading): 1 limit, 2 partial
 * cancel, 3 delete, 4 market (immediate-or-cancel, no price limit), 5 execution of a
 * named resting order (a replayed execution), 6 a message the book ignores (a replayed
 * hidden execution, cross trade or trading halt). */
void process(Book &bk, const Msg &m, TradeSink &ts, int32_t seq, int32_t t) {
    int64_t *ctr = ts.counters;
    ctr[C_MSGS] += 1;
    switch (m.type) {
    case LIMIT: {
        if (m.qty <= 0) { ctr[C_BAD] += 1; return; }
        int32_t q = match(bk, m, false, ts, seq, t);
        if (q <= 0) return;
        Side &own = bk.side(m.side);
        Order o{m.price, q, m.oid, m.tid, m.tsec, m.tns};
        if (own.count < bk.cap) {
            own.insert(o);
            return;
        }
        /* Reading: a full side evicts its worst order when the newcomer's price is
         * strictly better than that order's price; otherwise the remainder is dropped. */
        Order &w = own.worst();
        bool better = m.side == BUY ? m.price > w.price : m.price < w.price;
        if (better) {
            ctr[C_EVICT] += 1;
            ctr[C_EVICTED_QTY] += w.qty;
            own.pop_worst();
            own.insert(o);
        } else {
            ctr[C_DROP] += 1;
            ctr[C_DROPPED_QTY] += q;
        }
        return;
    }
    case MARKET: {
        if (m.qty <= 0) { ctr[C_BAD] += 1; return; }
        int32_t q = match(bk, m, true, ts, seq, t);
        ctr[C_MARKET_UNFILLED] += q;
        return;
    }
    case PARTIAL_CANCEL:
    case DELETE: {
        if (m.type == PARTIAL_CANCEL && m.qty <= 0) { ctr[C_BAD] += 1; return; }
        /* Reading: a cancel names the order by id on the message's side; a missing id
         * is a counted no-op; a partial cancel keeps the order's time priority. */
        Side &sd = bk.side(m.side);
        int64_t lk;
        size_t pos;
        Order *o = sd.find(m.oid, &lk, &pos);
        if (!o) { ctr[C_MISS] += 1; return; }
        if (m.type == DELETE) {
            sd.erase(lk, pos);
        } else {
            o->qty -= std::min(m.qty, o->qty);
            if (o->qty == 0) sd.erase(lk, pos);
        }
        return;
    }
    case EXECUTE: {
        /* Reading: a replayed execution names the resting order by id on the message's
         * side (the side of the executed order); it trades min(qty, the order's qty) at the
         * order's price against an anonymous aggressor of the other side (order id 0,
         * trader 0) and leaves the rest of the order with its priority.  A missing id is
         * a counted no-op, as for cancels. */
        if (m.qty <= 0) { ctr[C_BAD] += 1; return; }
        Side &sd = bk.side(m.side);
        int64_t lk;
        size_t pos;
        Order *o = sd.find(m.oid, &lk, &pos);
        if (!o) { ctr[C_MISS] += 1; return; }
        const int32_t x = std::min(m.qty, o->qty);
        const int32_t rec[TRADE_WORDS] = {o->price, x, 0, o->oid, 0, o->tid, (1 - m.side) | (seq << 1), t};
        emit_record(ts, rec);
        o->qty -= x;
        if (o->qty == 0) sd.erase(lk, pos);
        return;
    }
    case IGNORED:
        ctr[C_IGNORED] += 1;
        return;
    default:
        ctr[C_BAD] += 1;
        return;
    }
}

Msg decode_msg(const int32_t *w) {
    return Msg{w[0] & 0xFF, (w[0] >> 8) & 1, w[1], w[2], w[3], w[4], w[5], w[6]};
}

/* ------------------------------------------------------------------------------
 * Environments
 * ---------------------------------------------------------------------------- */
struct Agent {
    int64_t inv = 0, cash = 0, rem = 0, ctr = 0;
    int64_t step_bq = 0, step_sq = 0; /* bought / sold in the last step */
};

struct Env {
    Book book;
    int32_t last_bb = 0, last_ba = 0;
    int64_t mid2_prev = 0, p_init2 = 0, last_dmid2 = 0;
    int32_t last_tsec = 0, last_tns = 0;
    int32_t t = 0;
    int64_t counters[N_COUNTERS] = {};
    std::vector<Agent> agents;
    /* statistics of the last step (observation features) */
    int64_t st_buy_vol = 0, st_sell_vol = 0, st_trades = 0;
    int32_t st_last_price = 0;
    explicit Env(int32_t cap) : book(cap) {}
};

struct Desire {
    int side;
    int32_t price;
    int64_t qty;
};

int n_actions(int kind) {
    if (kind == AG_DIR) return 3;
    if (kind == AG_EXEC_TWAP || kind == AG_MM_AS) return 1; /* baselines: the action is not used */
    return 9;
}

/* floor(x / 2) and ceil(x / 2) for any sign */
int64_t floor_half(int64_t x) { return x >= 0 ? x / 2 : -((-x + 1) / 2); }
int64_t ceil_half2(int64_t x) { return -floor_half(-x); }

int64_t ceil_half(int64_t x) { return x >= 0 ? (x + 1) / 2 : -((-x) / 2); }

/* Sec. 4.1.2, execution agent (sell task): choose the price of an order of an a-priori
 * quantity q0; the "complex" variant adds 2x and 5x quantities.  Reading of the
 * reference prices: far touch bb, mid, near touch ba, deeper ba+2; action 8 ladders
 * four orders at ba..ba+3.  Orders are clipped in listed order to the remaining task. */
void decode_exec(int a, int32_t bb, int32_t ba, int64_t rem, int32_t q0, std::vector<Desire> &lim,
                 std::vector<Desire> &mkt) {
    std::vector<Desire> want;
    bool market = false;
    switch (a) {
    case 1: market = true; want.push_back({SELL, 0, q0}); break;
    case 2: want.push_back({SELL, bb, q0}); break;
    case 3: want.push_back({SELL, (int32_t)ceil_half((int64_t)bb + ba), q0}); break;
    case 4: want.push_back({SELL, ba, q0}); break;
    case 5: want.push_back({SELL, ba + 2, q0}); break;
    case 6: want.push_back({SELL, ba, 2 * (int64_t)q0}); break;
    case 7: want.push_back({SELL, ba, 5 * (int64_t)q0}); break;
    case 8:
        for (int k = 0; k < 4; ++k) want.push_back({SELL, ba + k, q0});
        break;
    default: break;
    }
    int64_t left = rem;
    for (auto d : want) {
        d.qty = std::min(d.qty, left);
        left -= d.qty;
        if (d.qty <= 0) continue;
        (market ? mkt : lim).push_back(d);
    }
}

/* Sec. 4.1.1, market maker, fixed-quantity action space with its eight options:
 * (i) no quotes, (ii)/(iii) 2 / 4 ticks from the best prices, (iv) one tick into the
 * spread, (v)/(vi) one side only, 2 ticks away, (vii)/(viii) 5 ticks away on one side
 * and one tick into the spread on the other.  Action 8 (reading) quotes a ladder of four
 * levels per side at offsets 0..3.  Bids never reach the step-start best ask and asks
 * never reach the step-start best bid. */
void decode_mm(int a, int32_t bb, int32_t ba, int32_t q, std::vector<Desire> &lim) {
    auto bid = [&](int o) { lim.push_back({BUY, std::min(bb - o, ba - 1), q}); };
    auto ask = [&](int o) { lim.push_back({SELL, std::max(ba + o, bb + 1), q}); };
    switch (a) {
    case 1: bid(2); ask(2); break;
    case 2: bid(4); ask(4); break;
    case 3: bid(-1); ask(-1); break;
    case 4: bid(2); break;
    case 5: ask(2); break;
    case 6: bid(5); ask(-1); break;
    case 7: bid(-1); ask(5); break;
    case 8:
        for (int o = 0; o < 4; ++o) bid(o);
        for (int o = 0; o < 4; ++o) ask(o);
        break;
    default: break;
    }
}

/* Sec. 4.1.1, market maker, Spread-Skew action space: tabular (spread, skew) pairs in
 * place of continuous spread and skew parameters.  Reading (the paper gives no table):
 * always two-sided (the space has no "no quote" option), spread S in {1, 3, 5} ticks
 * around the mid and skew k in {-1, 0, +1} ticks, action a = 3 * (index of S) + (index of
 * k): bid = floor((bb + ba - S) / 2) + k, ask = ceil((bb + ba + S) / 2) + k, then as for
 * the fixed-quantity space bids stay below the step-start best ask and asks above the
 * best bid. */
void decode_spread_skew(int a, int32_t bb, int32_t ba, int32_t q, std::vector<Desire> &lim) {
    static const int S[3] = {1, 3, 5};
    const int spread = S[a / 3], skew = a % 3 - 1;
    const int64_t m2 = (int64_t)bb + ba;
    const int64_t bid = floor_half(m2 - spread) + skew;
    const int64_t ask = ceil_half2(m2 + spread) + skew;
    lim.push_back({BUY, (int32_t)std::min<int64_t>(bid, (int64_t)ba - 1), q});
    lim.push_back({SELL, (int32_t)std::max<int64_t>(ask, (int64_t)bb + 1), q});
}

/* Sec. 4.1.1, market maker, AvSt action space: the Avellaneda-Stoikov quotes (reservation
 * price r = s - q gamma sigma^2 (T - t), spread gamma sigma^2 (T - t) + (2 / gamma)
 * ln(1 + gamma / kappa)) with the risk aversion gamma as the agent's choice.  Reading:
 * gamma_a = gamma0 * 2^(a - 4) for a = 0..8; s the step-start mid; q the inventory in quote
 * lots (inventory / mm_q); T - t the steps left in the episode including this one;
 * sigma^2 in ticks^2 per step and kappa per tick from the configuration; bid = floor(r -
 * spread / 2), ask = ceil(r + spread / 2), one quote per side of mm_q, clamped as the
 * fixed-quantity space.  Evaluated in double left to right; the ln term depends only on
 * the configuration and the action and is tabled once. */
struct AvstTable { double A[9], B[9]; };
AvstTable avst_table(const or_config &c) {
    AvstTable t{};
    for (int a = 0; a < 9; ++a) {
        const double g = (double)c.avst_gamma * std::ldexp(1.0, a - 4);
        t.A[a] = g * (double)c.avst_sigma2;
        t.B[a] = (2.0 / g) * std::log(1.0 + g / (double)c.avst_kappa);
    }
    return t;
}
int32_t clamp_price(double x) {
    const double lim = 1073741824.0; /* 2^30 */
    return (int32_t)(x < -lim ? -lim : (x > lim ? lim : x));
}
void decode_avst(int a, int32_t bb, int32_t ba, int64_t inv, int32_t steps_left, const or_config &c,
                 const AvstTable &tab, std::vector<Desire> &lim) {
    const double q = (double)inv / (double)c.mm_q;
    const double tau = (double)steps_left;
    const double mid = (double)((int64_t)bb + ba) * 0.5;
    const double r = mid - q * tab.A[a] * tau;
    const double d = tab.A[a] * tau + tab.B[a];
    const int32_t bid = clamp_price(std::floor(r - d * 0.5));
    const int32_t ask = clamp_price(std::ceil(r + d * 0.5));
    lim.push_back({BUY, (int32_t)std::min<int64_t>(bid, (int64_t)ba - 1), c.mm_q});
    lim.push_back({SELL, (int32_t)std::max<int64_t>(ask, (int64_t)bb + 1), c.mm_q});
}

/* Sec. 5.2.2, the TWAP baseline of the execution task.  Reading: the sell task follows a
 * linear schedule, ceil(task * (t + 1) / T) shares executed by the end of step t; each
 * step the agent sells the shortfall (at most its remainder) with one limit order at the
 * step-start best bid (aggressive: it takes the bid, and whatever does not fill rests
 * there). */
void decode_twap(int32_t bb, int64_t rem, int64_t task, int32_t t, int32_t T, std::vector<Desire> &lim) {
    const int64_t target = (task * (int64_t)(t + 1) + T - 1) / T;
    const int64_t done = task - rem;
    const int64_t q = std::min(std::max<int64_t>(target - done, 0), rem);
    if (q > 0) lim.push_back({SELL, bb, q});
}

/* Sec. 4.1.3, directional trading: a bid or an ask at the best price, or nothing.
 * Reading: "best price" is the opposite touch (the order takes liquidity). */
void decode_dir(int a, int32_t bb, int32_t ba, int32_t q, std::vector<Desire> &lim) {
    if (a == 1) lim.push_back({BUY, ba, q});
    if (a == 2) lim.push_back({SELL, bb, q});
}

struct Oracle {
    or_config cfg;
    std::vector<int32_t> caps, kinds, ids;
    std::vector<Env> envs;
    AvstTable avst{};
    bool was_reset = false;
};

void reset_env(Env &env, const Oracle &O, int e, const int32_t *const *f, const int32_t *n) {
    const int32_t mc = O.cfg.max_cap;
    for (int s = 0; s < 2; ++s) {
        int32_t cnt = std::min(std::max(n[e * 2 + s], 0), env.book.cap);
        std::vector<Order> v;
        int64_t base = ((int64_t)e * 2 + s) * mc;
        for (int32_t j = 0; j < cnt; ++j)
            v.push_back(Order{f[0][base + j], f[1][base + j], f[2][base + j], f[3][base + j],
                              f[4][base + j], f[5][base + j]});
        env.book.side(s).load(v);
    }
    /* Reading: an empty side falls back to one tick beyond the other side's best price
     * (0 when both are empty). */
    Side &b = env.book.bids, &a = env.book.asks;
    env.last_bb = !b.empty() ? b.best().price : (!a.empty() ? a.best().price - 1 : 0);
    env.last_ba = !a.empty() ? a.best().price : (!b.empty() ? b.best().price + 1 : 0);
    env.p_init2 = (int64_t)env.last_bb + env.last_ba;
    env.mid2_prev = env.p_init2;
    env.last_dmid2 = 0;
    /* Agent messages carry the time of the last processed message; at reset that is the
     * latest time in the snapshot. */
    env.last_tsec = 0;
    env.last_tns = 0;
    for (int s = 0; s < 2; ++s)
        for (const Order &o : env.book.side(s).list())
            if (o.tsec > env.last_tsec || (o.tsec == env.last_tsec && o.tns > env.last_tns)) {
                env.last_tsec = o.tsec;
                env.last_tns = o.tns;
            }
    env.t = 0;
    std::fill(std::begin(env.counters), std::end(env.counters), 0);
    env.agents.assign((size_t)O.cfg.n_agents, Agent{});
    for (int i = 0; i < O.cfg.n_agents; ++i)
        if (is_exec(O.kinds[(size_t)i])) env.agents[(size_t)i].rem = O.cfg.exec_task;
    env.st_buy_vol = env.st_sell_vol = env.st_trades = 0;
    env.st_last_price = 0;
}

/* Observation of agent i after the last step (40 features, all integer-valued,
 * converted to float with round-to-nearest-even).  Reading: the paper's observations
 * are "statistics related to the agents' task, such as the size of their current
 * inventory" (Sec. 4.1.1); the feature list is a reading of that passage. */
void observe(const Oracle &O, const Env &env, int i, float *out) {
    int64_t f[OBS_DIM] = {};
    const int32_t bb = env.last_bb, ba = env.last_ba;
    const int64_t mid2 = (int64_t)bb + ba;
    const int32_t tid = i + 1;
    const Agent &ag = env.agents[(size_t)i];
    f[0] = (int64_t)ba - bb;
    f[1] = env.last_dmid2;
    f[2] = mid2 - env.p_init2;
    int64_t own_bid = 0, own_ask = 0, own_n = 0;
    for (int s = 0; s < 2; ++s) {
        std::vector<Order> v = const_cast<Env &>(env).book.side(s).list();
        for (const Order &o : v) {
            int64_t d = s == BUY ? (int64_t)bb - o.price : (int64_t)o.price - ba;
            if (d >= 0 && d <= 9) f[(s == BUY ? 3 : 13) + d] += o.qty;
            f[s == BUY ? 23 : 24] += o.qty;
            f[s == BUY ? 25 : 26] += 1;
            if (o.tid == tid) {
                (s == BUY ? own_bid : own_ask) += o.qty;
                own_n += 1;
            }
        }
    }
    f[27] = env.st_buy_vol;
    f[28] = env.st_sell_vol;
    f[29] = env.st_trades;
    f[30] = env.st_trades > 0 ? 2 * (int64_t)env.st_last_price - mid2 : 0;
    f[31] = ag.inv;
    f[32] = ag.cash;
    f[33] = is_exec(O.kinds[(size_t)i]) ? ag.rem : 0;
    f[34] = (int64_t)O.cfg.episode_len - env.t;
    f[35] = own_bid;
    f[36] = own_ask;
    f[37] = own_n;
    f[38] = ag.step_bq;
    f[39] = ag.step_sq;
    for (int k = 0; k < OBS_DIM; ++k) out[k] = (float)f[k];
}

struct StepIO {
    int32_t n_steps;
    const int32_t *mf[7];
    const int64_t *off;
    int32_t off_steps;
    const int32_t *actions;
    int32_t *trades;
    const int64_t *trade_off;
    int32_t *n_trades;
    int64_t *fills;
    float *reward, *obs;
    uint8_t *done;
    int32_t *actions_out;
};

/* One env-step of env e (Sec. 4, steps 1-5). */
void env_step(Oracle &O, int e, int s, const StepIO &io, TradeSink &sink) {
    Env &env = O.envs[(size_t)e];
    const int A = O.cfg.n_agents;
    const int N = O.cfg.n_envs;
    const int32_t t = env.t;
    const uint64_t eid = (uint64_t)O.ids[(size_t)e]; /* env index in the hash keys */
    Book &bk = env.book;

    /* Reading: agents see the book as it stands at the start of the step; an empty side
     * falls back to the last known best price. */
    const int32_t bb0 = !bk.bids.empty() ? bk.bids.best().price : env.last_bb;
    const int32_t ba0 = !bk.asks.empty() ? bk.asks.best().price : env.last_ba;

    /* Step 1: action conversion.  Agents act in index order. */
    std::vector<Msg> cancels, actions;
    for (int i = 0; i < A; ++i) {
        const int kind = O.kinds[(size_t)i];
        Agent &ag = env.agents[(size_t)i];
        int a;
        if (io.actions) {
            a = io.actions[((int64_t)s * A + i) * N + e];
        } else {
            /* random policy: Lemire's multiply-shift of a 32-bit hash onto [0, n) */
            uint32_t u = (uint32_t)(chain_hash(O.cfg.seed, DOM_ACTION, eid, (uint64_t)t, (uint64_t)i) >> 32);
            a = (int)(((uint64_t)u * (uint64_t)n_actions(kind)) >> 32);
        }
        if (io.actions_out) io.actions_out[((int64_t)s * A + i) * N + e] = a;
        if (a < 0 || a >= n_actions(kind)) a = 0; /* out-of-range actions do nothing */

        std::vector<Desire> lim, mkt;
        if (kind == AG_EXEC) decode_exec(a, bb0, ba0, ag.rem, O.cfg.exec_q0, lim, mkt);
        else if (kind == AG_MM || kind == AG_MM_BUYSELL) decode_mm(a, bb0, ba0, O.cfg.mm_q, lim);
        else if (kind == AG_MM_SPREADSKEW) decode_spread_skew(a, bb0, ba0, O.cfg.mm_q, lim);
        else if (kind == AG_MM_AVST) decode_avst(a, bb0, ba0, ag.inv, O.cfg.episode_len - t, O.cfg, O.avst, lim);
        else if (kind == AG_MM_AS) decode_avst(4, bb0, ba0, ag.inv, O.cfg.episode_len - t, O.cfg, O.avst, lim);
        else if (kind == AG_EXEC_TWAP) decode_twap(bb0, ag.rem, O.cfg.exec_task, t, O.cfg.episode_len, lim);
        else decode_dir(a, bb0, ba0, O.cfg.dir_q, lim);
        /* desired quantity per (side, price), in order of first appearance */
        std::vector<Desire> levels;
        for (const Desire &d : lim) {
            bool found = false;
            for (Desire &l : levels)
                if (l.side == d.side && l.price == d.price) { l.qty += d.qty; found = true; }
            if (!found) levels.push_back(d);
        }
        auto desired = [&](int side, int32_t price) -> int64_t {
            for (const Desire &l : levels)
                if (l.side == side && l.price == price) return l.qty;
            return 0;
        };
        /* The agent's resting orders in book order (bids, then asks). */
        const int32_t tid = i + 1;
        struct Own { int side; Order o; };
        std::vector<Own> own;
        for (int sd = 0; sd < 2; ++sd)
            for (const Order &o : bk.side(sd).list())
                if (o.tid == tid) own.push_back({sd, o});
        auto resting = [&](int side, int32_t price) -> int64_t {
            int64_t r = 0;
            for (const Own &w : own)
                if (w.side == side && w.o.price == price) r += w.o.qty;
            return r;
        };
        /* Sec. 4 step 1: unmatched orders from earlier steps are cancelled unless the new
         * messages are at the same price level.  Reading: at a kept level the agent keeps
         * its queue position and trades only the difference to the desired quantity;
         * an excess is taken from its newest orders there. */
        std::vector<std::pair<std::pair<int, int32_t>, int64_t>> older; /* level -> qty seen */
        for (const Own &w : own) {
            const int64_t D = desired(w.side, w.o.price);
            const int64_t R = resting(w.side, w.o.price);
            int64_t seen = 0;
            bool have = false;
            for (auto &p : older)
                if (p.first.first == w.side && p.first.second == w.o.price) { seen = p.second; p.second += w.o.qty; have = true; }
            if (!have) older.push_back({{w.side, w.o.price}, w.o.qty});
            Msg c{0, w.side, w.o.price, 0, w.o.oid, tid, env.last_tsec, env.last_tns};
            if (D == 0) {
                c.type = DELETE;
                c.qty = w.o.qty;
                cancels.push_back(c);
            } else if (R > D) {
                const int64_t need = R - D;
                const int64_t newer = R - seen - w.o.qty;
                const int64_t x = std::min<int64_t>(std::max<int64_t>(need - newer, 0), w.o.qty);
                if (x > 0) {
                    c.type = PARTIAL_CANCEL;
                    c.qty = (int32_t)x;
                    cancels.push_back(c);
                }
            }
        }
        auto new_order = [&](int type, int side, int32_t price, int64_t qty) {
            int32_t oid = (int32_t)((1u << 30) | ((uint32_t)i << 26) | (uint32_t)(ag.ctr & ((1 << 26) - 1)));
            ag.ctr += 1;
            actions.push_back(Msg{type, side, price, (int32_t)qty, oid, tid, env.last_tsec, env.last_tns});
        };
        for (const Desire &l : levels) {
            int64_t R = resting(l.side, l.price);
            if (l.qty > R) new_order(LIMIT, l.side, l.price, l.qty - R);
        }
        for (const Desire &d : mkt) new_order(MARKET, d.side, 0, d.qty);
    }

    /* Step 2: random shuffle of the agents' new orders.  Reading: the permutation sorts
     * by a 32-bit counter hash of (seed, env, step, position), ties by position; the
     * cancels are left in agent order (they commute with each other). */
    std::vector<std::pair<uint64_t, Msg>> keyed;
    for (size_t k = 0; k < actions.size(); ++k) {
        uint32_t h = (uint32_t)(chain_hash(O.cfg.seed, DOM_SHUFFLE, eid, (uint64_t)t, (uint64_t)k) >> 32);
        keyed.push_back({((uint64_t)h << 32) | (uint64_t)k, actions[k]});
    }
    std::sort(keyed.begin(), keyed.end(),
              [](const std::pair<uint64_t, Msg> &x, const std::pair<uint64_t, Msg> &y) { return x.first < y.first; });

    /* Step 3: concatenate [cancels, shuffled actions, replay messages], in this order. */
    std::vector<Msg> seqv(cancels);
    for (auto &kv : keyed) seqv.push_back(kv.second);
    const int64_t *row = io.off + (int64_t)e * (io.off_steps + 1);
    for (int64_t j = row[t]; j < row[t + 1]; ++j) {
        int32_t w[7] = {io.mf[0][j], io.mf[1][j], io.mf[2][j], io.mf[3][j], io.mf[4][j], io.mf[5][j], io.mf[6][j]};
        seqv.push_back(decode_msg(w));
    }

    /* Step 4: the book processes the sequence; trades are recorded.  Mid statistics for
     * the reward: after each message with both sides non-empty, add bb + ba. */
    std::vector<int32_t> step_trades;
    sink.step = &step_trades;
    int64_t mid_sum = 0, mid_n = 0;
    for (size_t k = 0; k < seqv.size(); ++k) {
        process(bk, seqv[k], sink, (int32_t)k, t);
        env.last_tsec = seqv[k].tsec;
        env.last_tns = seqv[k].tns;
        if (bk.both()) {
            mid_sum += (int64_t)bk.bids.best().price + bk.asks.best().price;
            mid_n += 1;
        }
    }
    sink.step = nullptr;

    /* Step 5: outcomes.  Fills: a trade fills agent i as aggressor or as resting side. */
    std::vector<int64_t> bq((size_t)A, 0), bn((size_t)A, 0), sq((size_t)A, 0), sn((size_t)A, 0);
    int64_t buy_vol = 0, sell_vol = 0;
    int32_t last_price = 0;
    for (size_t r = 0; r < step_trades.size(); r += TRADE_WORDS) {
        const int32_t *x = step_trades.data() + r;
        const int32_t p = x[0], q = x[1], agg_tid = x[4], pas_tid = x[5], agg_side = x[6] & 1;
        (agg_side == BUY ? buy_vol : sell_vol) += q;
        last_price = p;
        for (int i = 0; i < A; ++i) {
            const int32_t tid = i + 1;
            if (agg_tid == tid) {
                if (agg_side == BUY) { bq[(size_t)i] += q; bn[(size_t)i] += (int64_t)p * q; }
                else { sq[(size_t)i] += q; sn[(size_t)i] += (int64_t)p * q; }
            }
            if (pas_tid == tid) {
                if (agg_side == BUY) { sq[(size_t)i] += q; sn[(size_t)i] += (int64_t)p * q; }
                else { bq[(size_t)i] += q; bn[(size_t)i] += (int64_t)p * q; }
            }
        }
    }
    const int64_t n_step_trades = (int64_t)step_trades.size() / TRADE_WORDS;

    /* reference prices at the end of the step */
    const int32_t bb1 = !bk.bids.empty() ? bk.bids.best().price : env.last_bb;
    const int32_t ba1 = !bk.asks.empty() ? bk.asks.best().price : env.last_ba;
    const int64_t mid2_end = (int64_t)bb1 + ba1;
    const bool last = (t + 1 == O.cfg.episode_len);

    for (int i = 0; i < A; ++i) {
        Agent &ag = env.agents[(size_t)i];
        const int kind = O.kinds[(size_t)i];
        ag.inv += bq[(size_t)i] - sq[(size_t)i];
        ag.cash += sn[(size_t)i] - bn[(size_t)i];
        if (is_exec(kind)) ag.rem -= sq[(size_t)i];
        ag.step_bq = bq[(size_t)i];
        ag.step_sq = sq[(size_t)i];
        /* Rewards: one double expression per agent kind, evaluated left to right, then
         * rounded once to float. */
        const double mbar = mid_n > 0 ? (double)mid_sum / (2.0 * (double)mid_n) : (double)env.mid2_prev * 0.5;
        const double mt = (double)mid2_end * 0.5;
        const double mprev = (double)env.mid2_prev * 0.5;
        const double psi_b = mbar * (double)bq[(size_t)i] - (double)bn[(size_t)i];
        const double psi_s = (double)sn[(size_t)i] - mbar * (double)sq[(size_t)i];
        double r;
        if (is_spooner(kind)) {
            /* Eq. 3 (Spooner): spread PnL plus inventory PnL, positive inventory PnL
             * weighted by lambda, minus the quadratic inventory penalty rho * I^2. */
            const double psi_inv = (double)ag.inv * (mt - mprev);
            const double pos = psi_inv > 0.0 ? psi_inv : 0.0;
            r = psi_b + psi_s + psi_inv - (1.0 - (double)O.cfg.mm_lambda) * pos -
                (double)O.cfg.mm_rho * ((double)ag.inv * (double)ag.inv);
        } else if (kind == AG_MM_BUYSELL) {
            /* the market maker rewarded by Eq. 4 (buy-sell), minus the quadratic
             * inventory penalty rho * I^2 */
            r = psi_b + psi_s - (double)O.cfg.mm_rho * ((double)ag.inv * (double)ag.inv);
        } else if (kind == AG_DIR) {
            /* Eq. 4 (buy-sell) */
            r = psi_b + psi_s;
        } else {
            /* Eq. 2 (slippage of the sell task against the price at reset), per step,
             * with the end-of-episode penalty on the unfilled remainder. */
            const double pinit = (double)env.p_init2 * 0.5;
            r = (double)sn[(size_t)i] - pinit * (double)sq[(size_t)i];
            if (last) r = r - ((double)O.cfg.exec_penalty * (double)ag.rem) * pinit;
        }
        io.reward[((int64_t)s * A + i) * N + e] = (float)r;
        int64_t *fl = io.fills + (((int64_t)s * A + i) * N + e) * 4;
        fl[0] = bq[(size_t)i];
        fl[1] = bn[(size_t)i];
        fl[2] = sq[(size_t)i];
        fl[3] = sn[(size_t)i];
    }

    env.st_buy_vol = buy_vol;
    env.st_sell_vol = sell_vol;
    env.st_trades = n_step_trades;
    env.st_last_price = last_price;
    env.last_dmid2 = mid2_end - env.mid2_prev;
    env.last_bb = bb1;
    env.last_ba = ba1;
    env.mid2_prev = mid2_end;
    env.t = t + 1;
    io.n_trades[(int64_t)s * N + e] = (int32_t)n_step_trades;
    io.done[(int64_t)s * N + e] = last ? 1 : 0;
    for (int i = 0; i < A; ++i) observe(O, env, i, io.obs + (((int64_t)s * A + i) * N + e) * OBS_DIM);
}

} // namespace

extern "C" {

uint64_t oe_hash(uint64_t seed, uint64_t dom, uint64_t a, uint64_t b, uint64_t c) {
    return chain_hash(seed, dom, a, b, c);
}

uint64_t oe_mix(uint64_t z) { return splitmix64_mix(z); }

void *ob_new(int32_t cap) { return new Book(cap); }
void ob_free(void *b) { delete static_cast<Book *>(b); }

int32_t ob_process(void *b, const int32_t *msg, int32_t seq, int32_t t, int32_t *trades,
                   int32_t max_trades, int64_t *counters) {
    TradeSink ts;
    ts.buf = trades;
    ts.cap = max_trades;
    ts.counters = counters;
    process(*static_cast<Book *>(b), decode_msg(msg), ts, seq, t);
    return (int32_t)ts.written;
}

int32_t ob_export(void *b, int32_t side, int32_t *out, int32_t max_n) {
    std::vector<Order> v = static_cast<Book *>(b)->side(side).list();
    int32_t n = 0;
    for (const Order &o : v) {
        if (n >= max_n) break;
        int32_t *r = out + (int64_t)n * 6;
        r[0] = o.price; r[1] = o.qty; r[2] = o.oid; r[3] = o.tid; r[4] = o.tsec; r[5] = o.tns;
        ++n;
    }
    return (int32_t)v.size();
}

void ob_load(void *b, int32_t side, const int32_t *in, int32_t n) {
    std::vector<Order> v;
    for (int32_t j = 0; j < n; ++j) {
        const int32_t *r = in + (int64_t)j * 6;
        v.push_back(Order{r[0], r[1], r[2], r[3], r[4], r[5]});
    }
    static_cast<Book *>(b)->side(side).load(v);
}

void *oe_new(const or_config *cfg) {
    if (!cfg || cfg->n_envs <= 0 || cfg->n_agents < 0 || cfg->n_agents > 4 || cfg->max_cap <= 0 ||
        cfg->episode_len <= 0 || !cfg->cap)
        return nullptr;
    Oracle *O = new Oracle();
    O->cfg = *cfg;
    O->caps.assign(cfg->cap, cfg->cap + cfg->n_envs);
    for (int32_t c : O->caps)
        if (c < 1 || c > cfg->max_cap) { delete O; return nullptr; }
    if (cfg->n_agents > 0) O->kinds.assign(cfg->agent_kind, cfg->agent_kind + cfg->n_agents);
    bool avst = false;
    for (int32_t k : O->kinds) {
        if (k < AG_EXEC || k > AG_MM_AS) { delete O; return nullptr; }
        avst = avst || k == AG_MM_AVST || k == AG_MM_AS;
    }
    /* the Avellaneda-Stoikov quotes need gamma > 0, kappa > 0, sigma^2 >= 0 and a quote size */
    if (avst && !(cfg->avst_gamma > 0.f && cfg->avst_kappa > 0.f && cfg->avst_sigma2 >= 0.f &&
                  std::isfinite(cfg->avst_gamma) && std::isfinite(cfg->avst_kappa) && std::isfinite(cfg->avst_sigma2) &&
                  cfg->mm_q > 0)) {
        delete O;
        return nullptr;
    }
    if (avst) O->avst = avst_table(*cfg);
    for (int32_t e = 0; e < cfg->n_envs; ++e) O->ids.push_back(cfg->env_id ? cfg->env_id[e] : e);
    O->cfg.cap = nullptr;
    O->cfg.agent_kind = nullptr;
    O->cfg.env_id = nullptr;
    for (int32_t e = 0; e < cfg->n_envs; ++e) O->envs.emplace_back(O->caps[(size_t)e]);
    return O;
}

void oe_free(void *o) { delete static_cast<Oracle *>(o); }

int32_t oe_reset(void *o, const int32_t *price, const int32_t *qty, const int32_t *oid,
                 const int32_t *tid, const int32_t *tsec, const int32_t *tns, const int32_t *n) {
    Oracle &O = *static_cast<Oracle *>(o);
    const int32_t *f[6] = {price, qty, oid, tid, tsec, tns};
    for (int32_t e = 0; e < O.cfg.n_envs; ++e) reset_env(O.envs[(size_t)e], O, e, f, n);
    O.was_reset = true;
    return 0;
}

int32_t oe_step(void *o, int32_t n_steps, const int32_t *ts, const int32_t *price, const int32_t *qty,
                const int32_t *oid, const int32_t *tid, const int32_t *tsec, const int32_t *tns,
                const int64_t *off, int32_t off_steps, const int32_t *actions, int32_t *trades,
                const int64_t *trade_off, int32_t *n_trades, int64_t *fills, float *reward, float *obs,
                uint8_t *done, int32_t *actions_out, int32_t n_threads) {
    Oracle &O = *static_cast<Oracle *>(o);
    if (!O.was_reset) return -4;
    if (n_steps < 0) return -1;
    for (const Env &env : O.envs)
        if (env.t + n_steps > O.cfg.episode_len || env.t + n_steps > off_steps) return -4;
    StepIO io{n_steps, {ts, price, qty, oid, tid, tsec, tns}, off, off_steps, actions, trades, trade_off,
              n_trades, fills, reward, obs, done, actions_out};
    const int32_t N = O.cfg.n_envs;
    if (n_threads < 1) n_threads = 1;
    if (n_threads > N) n_threads = N;
    auto work = [&](int32_t e0, int32_t e1) {
        for (int32_t e = e0; e < e1; ++e) {
            TradeSink sink;
            sink.buf = trades ? trades + trade_off[e] * TRADE_WORDS : nullptr;
            sink.cap = trades ? trade_off[e + 1] - trade_off[e] : 0;
            sink.counters = O.envs[(size_t)e].counters;
            for (int32_t s = 0; s < n_steps; ++s) env_step(O, e, s, io, sink);
        }
    };
    std::vector<std::thread> th;
    for (int32_t k = 0; k < n_threads; ++k)
        th.emplace_back(work, (int32_t)((int64_t)N * k / n_threads), (int32_t)((int64_t)N * (k + 1) / n_threads));
    for (auto &x : th) x.join();
    return 0;
}

int32_t oe_observe(void *o, float *obs) {
    Oracle &O = *static_cast<Oracle *>(o);
    if (!O.was_reset) return -4;
    const int32_t N = O.cfg.n_envs, A = O.cfg.n_agents;
    for (int32_t e = 0; e < N; ++e)
        for (int32_t i = 0; i < A; ++i)
            observe(O, O.envs[(size_t)e], i, obs + ((int64_t)i * N + e) * OBS_DIM);
    return 0;
}

/* Books in the canonical layout: [n_envs][2][max_cap] per field, priority order,
 * unused slots zero; n is [n_envs][2]. */
int32_t oe_export_books(void *o, int32_t *price, int32_t *qty, int32_t *oid, int32_t *tid,
                        int32_t *tsec, int32_t *tns, int32_t *n) {
    Oracle &O = *static_cast<Oracle *>(o);
    const int32_t mc = O.cfg.max_cap;
    int32_t *f[6] = {price, qty, oid, tid, tsec, tns};
    for (int32_t e = 0; e < O.cfg.n_envs; ++e) {
        for (int s = 0; s < 2; ++s) {
            std::vector<Order> v = O.envs[(size_t)e].book.side(s).list();
            int64_t base = ((int64_t)e * 2 + s) * mc;
            for (int32_t j = 0; j < mc; ++j) {
                Order z{0, 0, 0, 0, 0, 0};
                const Order &x = j < (int32_t)v.size() ? v[(size_t)j] : z;
                f[0][base + j] = x.price; f[1][base + j] = x.qty; f[2][base + j] = x.oid;
                f[3][base + j] = x.tid; f[4][base + j] = x.tsec; f[5][base + j] = x.tns;
            }
            n[e * 2 + s] = (int32_t)v.size();
        }
    }
    return 0;
}

/* env_state [n_envs][12]: last_bb, last_ba, mid2_prev, p_init2, last_tsec, last_tns, t,
 * last_dmid2, then the last step's statistics (buyer- and seller-initiated volume, trades,
 * last trade price).  agent_state [n_envs][n_agents][6]: inventory, cash, remaining,
 * order counter, bought and sold in the last step.  counters [n_envs][11]. */
int32_t oe_export_state(void *o, int64_t *env_state, int64_t *agent_state, int64_t *counters) {
    Oracle &O = *static_cast<Oracle *>(o);
    const int32_t A = O.cfg.n_agents;
    for (int32_t e = 0; e < O.cfg.n_envs; ++e) {
        const Env &v = O.envs[(size_t)e];
        int64_t *es = env_state + (int64_t)e * ENV_WORDS;
        es[0] = v.last_bb; es[1] = v.last_ba; es[2] = v.mid2_prev; es[3] = v.p_init2;
        es[4] = v.last_tsec; es[5] = v.last_tns; es[6] = v.t; es[7] = v.last_dmid2;
        es[8] = v.st_buy_vol; es[9] = v.st_sell_vol; es[10] = v.st_trades; es[11] = v.st_last_price;
        for (int32_t i = 0; i < A; ++i) {
            int64_t *as = agent_state + ((int64_t)e * A + i) * AGENT_WORDS;
            const Agent &g = v.agents[(size_t)i];
            as[0] = g.inv; as[1] = g.cash; as[2] = g.rem; as[3] = g.ctr;
            as[4] = g.step_bq; as[5] = g.step_sq;
        }
        for (int k = 0; k < N_COUNTERS; ++k) counters[(int64_t)e * N_COUNTERS + k] = v.counters[k];
    }
    return 0;
}

/* The inverse of oe_export_books + oe_export_state: every env continues from the given
 * books (canonical layout, counts clamped to the capacity) and state, as if it had been
 * stepped there (Sec. 4: an episode starts from a book state).  The step counter of every
 * env is set to `step`; counters may be NULL (zero). */
int32_t oe_import_state(void *o, const int32_t *price, const int32_t *qty, const int32_t *oid,
                        const int32_t *tid, const int32_t *tsec, const int32_t *tns, const int32_t *n,
                        const int64_t *env_state, const int64_t *agent_state, const int64_t *counters,
                        int32_t step) {
    Oracle &O = *static_cast<Oracle *>(o);
    if (step < 0 || step > O.cfg.episode_len) return -1;
    const int32_t A = O.cfg.n_agents, mc = O.cfg.max_cap;
    const int32_t *f[6] = {price, qty, oid, tid, tsec, tns};
    for (int32_t e = 0; e < O.cfg.n_envs; ++e) {
        Env &v = O.envs[(size_t)e];
        for (int s = 0; s < 2; ++s) {
            const int32_t cnt = std::min(std::max(n[e * 2 + s], 0), v.book.cap);
            std::vector<Order> list;
            const int64_t base = ((int64_t)e * 2 + s) * mc;
            for (int32_t j = 0; j < cnt; ++j)
                list.push_back(Order{f[0][base + j], f[1][base + j], f[2][base + j], f[3][base + j],
                                     f[4][base + j], f[5][base + j]});
            v.book.side(s).load(list);
        }
        const int64_t *es = env_state + (int64_t)e * ENV_WORDS;
        v.last_bb = (int32_t)es[0]; v.last_ba = (int32_t)es[1]; v.mid2_prev = es[2]; v.p_init2 = es[3];
        v.last_tsec = (int32_t)es[4]; v.last_tns = (int32_t)es[5]; v.t = step; v.last_dmid2 = es[7];
        v.st_buy_vol = es[8]; v.st_sell_vol = es[9]; v.st_trades = es[10]; v.st_last_price = (int32_t)es[11];
        v.agents.assign((size_t)A, Agent{});
        for (int32_t i = 0; i < A; ++i) {
            const int64_t *as = agent_state + ((int64_t)e * A + i) * AGENT_WORDS;
            Agent &g = v.agents[(size_t)i];
            g.inv = as[0]; g.cash = as[1]; g.rem = as[2]; g.ctr = as[3];
            g.step_bq = as[4]; g.step_sq = as[5];
        }
        for (int k = 0; k < N_COUNTERS; ++k) v.counters[k] = counters ? counters[(int64_t)e * N_COUNTERS + k] : 0;
    }
    O.was_reset = true;
    return 0;
}

} // extern "C"
