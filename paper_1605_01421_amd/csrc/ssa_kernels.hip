// ssa_kernels.hip -- gfx950 kernels of the split-step direct-method SSA
// (section 2.3 and Appendix A of arXiv 1605.01421): one lane per node.
//
// Three persistent kernels per model, chosen by the host runtime:
//  * free_kernel (no external transfers): nodes are independent for the whole
//    run, so each wavefront takes 64-node chunks from a work queue and carries
//    every node through all days with its state in registers.
//  * flow_kernel (external transfers, every node resident): node state stays
//    in registers and transfers are applied peer to peer.  Each node walks its
//    own transfers in key order; as the source it samples the individuals,
//    removes them and posts the (shifted) counts to the transfer's mailbox
//    word; as the destination it waits for that word and adds the counts.
//    Only the per-node order matters for the result, so this equals the
//    serial order; nodes without transfers never wait, and there is no
//    grid-wide barrier.
//  * sync_kernel (external transfers, more nodes than resident lanes): all
//    lanes meet at a grid barrier on every day with transfers; workgroup 0
//    applies them level by level in global memory; a second barrier follows.
// The flow and sync kernels are launched cooperatively (all workgroups
// resident).  Every wait has a wall-clock limit that turns a stall into an
// error.
// The device part (everything up to the host launchers) is also compiled at
// run time with hipRTC for models generated from transition strings; the
// host part is left out there.
#include "device_math.h"
#include "internal.h"
#include "models.h"

#ifndef __HIPCC_RTC__
#include <algorithm>

#include "siminf.h"
#endif

namespace siminf {

namespace {

constexpr int E_NEG_STATE = -5, E_BAD_RATE = -6, E_OVERDRAW = -7, E_PTS = -9, E_STEP_LIMIT = -10;
constexpr int NO_STEP = 0x7fffffff;  // the day index of "no transfer item left"
constexpr int EV_EXIT = 0, EV_ENTER = 1, EV_EXTTRANS = 3;

// Implementation limit on the draws of one node within one unit of time (the
// method itself has none).  The draw index is the first Philox counter word,
// so a node-day has 2^32 distinct blocks; the library stops far earlier so
// that a node with exploding rates ends the run (E_STEP_LIMIT, keyed like any
// SSA error) instead of holding its lane for hours.  A node that needs the
// draw with index STEP_LIMIT fails; every node-day with fewer draws is the
// method's own result.
constexpr uint32_t STEP_LIMIT = 1u << 24;

__device__ __forceinline__ void raise_error(Ctrl* c, int step, int phase, int64_t ord, int code) {
    atomicMin(&c->err_key, make_err_key((uint32_t)step, (uint32_t)phase, (uint64_t)ord, (uint32_t)(-code)));
}

// Wall-clock limit of one wait: the constant-rate real-time counter is read
// every 256 polls; the first read starts the clock.
struct WaitClock {
    uint64_t start = 0;
    __device__ __forceinline__ bool expired(uint64_t limit) {
        const uint64_t now = (uint64_t)wall_clock64();
        if (start == 0) {
            start = now | 1ull;
            return false;
        }
        return now - start > limit;
    }
};

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, WAVE);
    return x;
}

__device__ __forceinline__ uint64_t load_error_step(Ctrl* c) {
    return __hip_atomic_load(&c->err_key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >> 44;
}

// First step whose error stops further work, read by lane 0 (wave-uniform).
__device__ __forceinline__ uint64_t error_step(Ctrl* c) {
    uint64_t k = 0;
    if ((threadIdx.x & (WAVE - 1)) == 0) k = load_error_step(c);
    return __shfl(k, 0, WAVE);
}

template <class M>
struct Node {
    int32_t u[M::NC];
    double v[M::NV > 0 ? M::NV : 1];
    double ld[M::NLD > 0 ? M::NLD : 1];
    double gd[M::NGD > 0 ? M::NGD : 1];
};

__device__ __forceinline__ bool rate_ok(double w) { return w >= 0.0 && isfinite(w); }

struct StepRandoms {
    double e;   // -log(r1): the Exp(1) variate of the waiting time
    double r2;  // uniform for the inversion search
};

__device__ __forceinline__ StepRandoms step_randoms(uint32_t k0, uint32_t k1, uint32_t step, uint32_t day,
                                                    uint32_t node, uint32_t tag) {
    const Block4 r = philox10(k0, k1, step, day, node, tag);
    return {-series_log(open_uniform(r.x, r.y)), open_uniform(r.z, r.w)};
}

template <class M>
struct Transition {
    int32_t u[M::NC];
    double w0, w1;
    int err;
};

// Inversion (first transition with positive rate whose cumulative sum
// reaches x = lambda*r2; the running sum after the first rate is w0), the
// state after adding column n of S, and the rates the dependency graph marks
// for recomputation.  err: E_NEG_STATE if a compartment went negative, else
// E_BAD_RATE if a recomputed rate is negative or not finite, else 0.
template <class M>
__device__ __forceinline__ Transition<M> transition_of(const KParams& p, const int32_t* u, const double* v,
                                                       const double* ld, const double* gd, double w0, double w1,
                                                       double x) {
    Transition<M> r;
    const int n = (w0 > 0.0 && x <= w0) ? 0 : (w1 > 0.0 ? 1 : 0);
    bool neg = false;
#pragma unroll
    for (int c = 0; c < M::NC; ++c) {
        r.u[c] = u[c] + (n ? p.S[c + M::NC] : p.S[c]);
        neg |= r.u[c] < 0;
    }
    const uint32_t g = n ? p.Gmask[1] : p.Gmask[0];
    r.w0 = (g & 1u) ? M::template rate<0>(r.u, v, ld, gd) : w0;
    r.w1 = (g & 2u) ? M::template rate<1>(r.u, v, ld, gd) : w1;
    r.err = neg ? E_NEG_STATE : (rate_ok(r.w0) && rate_ok(r.w1)) ? 0 : E_BAD_RATE;
    return r;
}

template <class M>
__device__ __forceinline__ Transition<M> transition(const KParams& p, const Node<M>& s, double w0, double w1,
                                                    double x) {
    return transition_of<M>(p, s.u, s.v, s.ld, s.gd, w0, w1, x);
}

// Direct-method SSA of a node of a generated model (any number of
// transitions; state changes, dependency graph and rates compiled into the
// model type).  The same steps as ssa_to_boundary in the same order, over
// NT rates: lambda as a left-to-right sum, the step limit before each draw,
// tau = -log(r1)/lambda, stop if t + tau >= T, inversion (the first
// transition with a positive rate whose running sum reaches lambda*r2, else
// the last with a positive rate), the transition's column of S, the
// negative-state check, and the rates its column of G marks.
template <class M>
__device__ __forceinline__ int ssa_generated(const KParams& p, Node<M>& s, double t, double T, uint32_t day_word,
                                             uint32_t node, uint32_t stream, unsigned long long& transitions,
                                             unsigned long long& draws) {
    double w[M::NT];
    bool bad = false;
#pragma unroll
    for (int j = 0; j < M::NT; ++j) {
        w[j] = M::rate(j, s.u, s.v, s.ld, s.gd);
        bad = bad || !rate_ok(w[j]);
    }
    if (bad) return E_BAD_RATE;
    const uint32_t k0 = (uint32_t)p.seed, k1 = (uint32_t)(p.seed >> 32);
    const uint32_t tag = stream & 0xFFFFFFu;
    for (uint32_t step = 0;; ++step) {
        double lam = 0.0;
#pragma unroll
        for (int j = 0; j < M::NT; ++j) lam = lam + w[j];
        if (!(lam > 0.0)) return 0;
        if (step == STEP_LIMIT) return E_STEP_LIMIT;
        const StepRandoms r = step_randoms(k0, k1, step, day_word, node, tag);
        draws += 1;
        const double tn = t + r.e / lam;
        if (tn >= T) return 0;
        t = tn;
        const double x = lam * r.r2;
        double cum = 0.0;
        int n = -1, last = -1;
#pragma unroll
        for (int j = 0; j < M::NT; ++j) {
            cum = cum + w[j];
            const bool pos = w[j] > 0.0;
            last = pos ? j : last;
            n = (n < 0 && pos && x <= cum) ? j : n;
        }
        if (n < 0) n = last;
        M::apply(n, s.u);
        transitions += 1;
        bool neg = false;
#pragma unroll
        for (int c = 0; c < M::NC; ++c) neg = neg || s.u[c] < 0;
        if (neg) return E_NEG_STATE;
        const uint32_t g = M::deps(n);
#pragma unroll
        for (int j = 0; j < M::NT; ++j)
            if ((g >> j) & 1u) {
                w[j] = M::rate(j, s.u, s.v, s.ld, s.gd);
                bad = bad || !rate_ok(w[j]);
            }
        if (bad) return E_BAD_RATE;
    }
}

// Direct-method SSA of one node from time t to the day boundary T
// (Appendix A): lambda = w0 + w1, tau = -log(r1)/lambda, stop if
// t + tau >= T, else pick the transition by inversion with r2, apply its
// column of S and recompute the rates marked in G.  With PIPE the random
// numbers of the next step (which do not depend on the state) are computed
// while the current step's dependent chain runs; the values are identical.
template <class M, bool PIPE>
__device__ __forceinline__ int ssa_to_boundary(const KParams& p, Node<M>& s, double t, double T,
                                               uint32_t day_word, uint32_t node, uint32_t stream,
                                               unsigned long long& transitions, unsigned long long& draws) {
    if constexpr (M::GENERATED) {
        return ssa_generated<M>(p, s, t, T, day_word, node, stream, transitions, draws);
    } else {
    static_assert(M::NT == 2, "the built-in models have two transitions");
    double w0 = M::template rate<0>(s.u, s.v, s.ld, s.gd);
    double w1 = M::template rate<1>(s.u, s.v, s.ld, s.gd);
    if (!rate_ok(w0) || !rate_ok(w1)) return E_BAD_RATE;
    const uint32_t k0 = (uint32_t)p.seed, k1 = (uint32_t)(p.seed >> 32);
    const uint32_t tag = stream & 0xFFFFFFu;
    double lam = 0.0;
    lam = lam + w0;
    lam = lam + w1;
    if (!(lam > 0.0)) return 0;
    StepRandoms cur = step_randoms(k0, k1, 0u, day_word, node, tag);
    for (uint32_t step = 0;;) {
        if (step == STEP_LIMIT) return E_STEP_LIMIT;
        draws += 1;
        StepRandoms nxt{0.0, 0.0};
        if constexpr (PIPE) nxt = step_randoms(k0, k1, step + 1u, day_word, node, tag);
        const double tau = cur.e / lam;
        const double tn = t + tau;
        // the transition, its state and the recomputed rates do not depend on
        // tau: they are computed alongside the division and kept only if the
        // step stays inside the day
        const Transition<M> nx = transition<M>(p, s, w0, w1, lam * cur.r2);
        if (tn >= T) break;
        t = tn;
#pragma unroll
        for (int c = 0; c < M::NC; ++c) s.u[c] = nx.u[c];
        w0 = nx.w0;
        w1 = nx.w1;
        transitions += 1;
        if (nx.err) return nx.err;
        lam = 0.0;
        lam = lam + w0;
        lam = lam + w1;
        if (!(lam > 0.0)) break;
        ++step;
        if constexpr (PIPE)
            cur = nxt;
        else
            cur = step_randoms(k0, k1, step, day_word, node, tag);
    }
    return 0;
    }
}

__device__ __forceinline__ double read_lane(double x, int lane) {
    const long long bits = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)bits, lane);
    const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// The same SSA for one node carried by a whole wavefront: every lane holds
// the node's state and runs the same dependent chain (so the state stays
// wave-uniform), while the random numbers, which do not depend on the state,
// are drawn 64 steps at a time with lane j computing step base + j.  Only
// lane 0 counts.  Bit-identical to ssa_to_boundary.
template <class M>
__device__ __forceinline__ int ssa_wide(const KParams& p, Node<M>& s, double t, double T, uint32_t day_word,
                                        uint32_t node, uint32_t stream, unsigned long long& transitions,
                                        unsigned long long& draws) {
    const int lane = threadIdx.x & (WAVE - 1);
    double w0 = M::template rate<0>(s.u, s.v, s.ld, s.gd);
    double w1 = M::template rate<1>(s.u, s.v, s.ld, s.gd);
    if (!rate_ok(w0) || !rate_ok(w1)) return E_BAD_RATE;
    const uint32_t k0 = (uint32_t)p.seed, k1 = (uint32_t)(p.seed >> 32);
    const uint32_t tag = stream & 0xFFFFFFu;
    double lam = 0.0;
    lam = lam + w0;
    lam = lam + w1;
    if (!(lam > 0.0)) return 0;
    const unsigned long long one = lane == 0 ? 1ull : 0ull;
    for (uint32_t base = 0;; base += WAVE) {
        if (base >= STEP_LIMIT) return E_STEP_LIMIT;
        const StepRandoms mine = step_randoms(k0, k1, base + (uint32_t)lane, day_word, node, tag);
        for (int i = 0; i < WAVE; ++i) {
            const double e = read_lane(mine.e, i);
            const double r2 = read_lane(mine.r2, i);
            draws += one;
            const double tau = e / lam;
            const double tn = t + tau;
            const Transition<M> nx = transition<M>(p, s, w0, w1, lam * r2);
            if (tn >= T) return 0;
            t = tn;
#pragma unroll
            for (int c = 0; c < M::NC; ++c) s.u[c] = nx.u[c];
            w0 = nx.w0;
            w1 = nx.w1;
            transitions += one;
            if (nx.err) return nx.err;
            lam = 0.0;
            lam = lam + w0;
            lam = lam + w1;
            if (!(lam > 0.0)) return 0;
        }
    }
}

// Steps per window of the lattice walk, the lanes its points occupy, and
// the draws of one block (a whole number of windows).
constexpr int LAT_W = 10;
constexpr int LAT_POINTS = LAT_W * (LAT_W + 1) / 2;
constexpr int LAT_BLOCK = 60;
static_assert(LAT_POINTS <= WAVE && LAT_BLOCK <= WAVE && LAT_BLOCK % LAT_W == 0, "the lattice must fit one wavefront");

// The points of a window's path: pl[k + 1] = pl[k] + k + 1 + (bit pl[k] of
// mask), each on the scalar unit as a bit test that sets SCC and an add with
// carry of the constant k + 1 (arithmetic only; SCC is set and used inside
// the block).
template <int K>
__device__ __forceinline__ void lattice_path(unsigned long long mask, int (&pl)[LAT_W + 1]) {
    if constexpr (K < LAT_W) {
        int r;
        asm("s_bitcmp1_b64 %1, %2\n\ts_addc_u32 %0, %2, %3" : "=s"(r) : "s"(mask), "s"(pl[K]), "n"(K + 1) : "scc");
        pl[K + 1] = r;
        lattice_path<K + 1>(mask, pl);
    }
}

// What one pass of the lattice walk gives a lane: the values of the step
// taken from its point, and the check of its state (1 a negative
// compartment, 2 a bad rate, 4 lambda <= 0: the node stops for the day).  A
// state that fails its checks is never left by a step, so its tau is +inf;
// a state that passes has lambda > 0 and a finite tau >= 0.  `first` has bit
// L set when the step from point L is of the first kind.
struct LatticePass {
    double tau, lam;
    int chk;
    unsigned long long first;
};

// Lane (lk, la) evaluates the state lk steps ahead of u with la transitions
// of the first kind, with the variates e, r2 of step lk.
template <class M>
__device__ __forceinline__ LatticePass lattice_pass(const Node<M>& s, const int32_t (&u)[M::NC], int lk, int la,
                                                    const int32_t (&S0)[M::NC], const int32_t (&S1)[M::NC],
                                                    double e, double r2) {
    int32_t uc[M::NC];
    bool neg = false;
#pragma unroll
    for (int c = 0; c < M::NC; ++c) {
        uc[c] = u[c] + la * S0[c] + (lk - la) * S1[c];
        neg |= uc[c] < 0;
    }
    const double c0 = M::template rate<0>(uc, s.v, s.ld, s.gd);
    const double c1 = M::template rate<1>(uc, s.v, s.ld, s.gd);
    LatticePass r;
    double lam = 0.0;
    lam = lam + c0;
    lam = lam + c1;
    r.lam = lam;
    const double x = lam * r2;
    const int n = (c0 > 0.0 && x <= c0) ? 0 : (c1 > 0.0 ? 1 : 0);
    r.chk = neg ? 1 : !(rate_ok(c0) && rate_ok(c1)) ? 2 : !(lam > 0.0) ? 4 : 0;
    r.tau = r.chk ? __builtin_inf() : e / lam;
    r.first = __ballot(n == 0);
    return r;
}

// The same SSA for one heavy node on a whole wavefront, with the serial chain
// cut to a few instructions per step.  With two transitions, the state k
// steps ahead is u + a S[:,0] + (k - a) S[:,1] for some 0 <= a <= k.  One
// wavefront-wide pass evaluates, for every lattice point (k, a) of the next
// LAT_W steps at once, all that a step computes from its state: the checks
// of the state, the rates, lambda, tau = E_k / lambda (E_k is the
// exponential variate of step k), and the inversion choice with r2_k.  The
// walk then follows the realised path: per step it reads tau from the lane
// of the current point and advances t by one addition, and it stops at the
// day boundary.  The path, and so the window's end state, is known before
// the time additions: the next window's pass is computed alongside them and
// used if the window does not stop.  Every value comes from the same
// operations in the same order as in ssa_to_boundary, so the result is
// bit-identical.  Valid when G marks both rates after either transition: a
// full recomputation then equals the incremental one.
template <class M>
__device__ __forceinline__ int ssa_lattice(const KParams& p, Node<M>& s, double t, double T, uint32_t day_word,
                                           uint32_t node, uint32_t stream, unsigned long long& transitions,
                                           unsigned long long& draws) {
    {
        // the day's first state, checked as the walk's first pass would (a
        // node whose rates are all zero costs no draw)
        bool neg = false;
#pragma unroll
        for (int c = 0; c < M::NC; ++c) neg |= s.u[c] < 0;
        if (neg) return E_NEG_STATE;
        const double w0 = M::template rate<0>(s.u, s.v, s.ld, s.gd);
        const double w1 = M::template rate<1>(s.u, s.v, s.ld, s.gd);
        if (!rate_ok(w0) || !rate_ok(w1)) return E_BAD_RATE;
        double lam = 0.0;
        lam = lam + w0;
        lam = lam + w1;
        if (!(lam > 0.0)) return 0;
    }
    const int lane = threadIdx.x & (WAVE - 1);
    int lk = 0;
    while ((lk + 1) * (lk + 2) / 2 <= lane) ++lk;
    const int la = lane - lk * (lk + 1) / 2;
    const uint32_t k0 = (uint32_t)p.seed, k1 = (uint32_t)(p.seed >> 32);
    const uint32_t tag = stream & 0xFFFFFFu;
    int32_t S0[M::NC], S1[M::NC], Sw[M::NC], Sd[M::NC];
#pragma unroll
    for (int c = 0; c < M::NC; ++c) {
        S0[c] = p.S[c];
        S1[c] = p.S[c + M::NC];
        Sw[c] = LAT_W * S1[c];  // a full window with a first-kind steps moves
        Sd[c] = S0[c] - S1[c];  // the state by Sw + a Sd
    }
    uint32_t nd = 0, ntr = 0;  // draws and transitions, wave-uniform
    int rc = 0;
    // Draws come in blocks of LAT_BLOCK (lane j of the block at mb draws step
    // mb + j); the window at draw g (a multiple of LAT_W) reads the lanes
    // g - mb + lk of its block.
    const int lsrc = lk < LAT_W ? lk : 0;
    uint32_t mb = 0;
    StepRandoms mine = step_randoms(k0, k1, (uint32_t)lane, day_word, node, tag);
    auto ensure_block = [&](uint32_t g) {
        if (g - mb >= (uint32_t)LAT_BLOCK) {
            mb = g;
            mine = step_randoms(k0, k1, g + (uint32_t)lane, day_word, node, tag);
        }
    };
    LatticePass P = lattice_pass<M>(s, s.u, lk, la, S0, S1, __shfl(mine.e, lsrc, WAVE), __shfl(mine.r2, lsrc, WAVE));
#pragma unroll 1
    for (uint32_t g = 0;; g += LAT_W) {
        const double t_in = t;
        const bool near_limit = g <= STEP_LIMIT && STEP_LIMIT - g < (uint32_t)LAT_W;
        // Fast path, taken by every window but the day's last: the path in
        // scalar registers, tau read from the lane of each point in turn.
        // The times only grow (every tau is >= 0), so a window that ends
        // before T neither crosses the boundary nor meets a failing state.
        // A window that starts less than twice its expected length before T
        // (or in a state without a positive rate) goes to the slow path at
        // once: it most likely stops there.
        if (!near_limit && (T - t) * read_lane(P.lam, 0) > 2.0 * LAT_W) {
            ensure_block(g + LAT_W);
            const int src = (int)(g + LAT_W - mb) + lsrc;
            const double en = __shfl(mine.e, src, WAVE);
            const double r2n = __shfl(mine.r2, src, WAVE);
            // point of step k; the path's last point is LAT_POINTS + a (every
            // step k adds k + 1, and 1 more if of the first kind)
            int pl[LAT_W + 1];
            pl[0] = 0;
            lattice_path<0>(P.first, pl);
            const int a = pl[LAT_W] - LAT_POINTS;
            int32_t un[M::NC];
#pragma unroll
            for (int c = 0; c < M::NC; ++c) un[c] = s.u[c] + Sw[c] + a * Sd[c];
            // the next window's pass, from the state this one ends in
            const LatticePass Pn = lattice_pass<M>(s, un, lk, la, S0, S1, en, r2n);
            double tv[LAT_W];
#pragma unroll
            for (int k = 0; k < LAT_W; ++k) tv[k] = read_lane(P.tau, pl[k]);
#pragma unroll
            for (int k = 0; k < LAT_W; ++k) t = t + tv[k];
            // the next pass is needed only if the window goes through; this
            // empty statement makes it be computed here, beside the time
            // additions, rather than after the test (no instruction)
            asm volatile("" ::"v"(Pn.tau), "v"(Pn.lam), "v"(Pn.chk));
            if (t < T) {
#pragma unroll
                for (int c = 0; c < M::NC; ++c) s.u[c] = un[c];
                nd += (uint32_t)LAT_W;
                ntr += (uint32_t)LAT_W;
                P = Pn;
                continue;
            }
            t = t_in;
        }
        // Slow path (the window that stops).  The window's first state (the
        // day's starting state or the one the previous window ended in) is
        // checked before its first draw.
        const int c00 = __builtin_amdgcn_readfirstlane(P.chk);
        if (c00) {
            rc = (c00 & 1) ? E_NEG_STATE : (c00 & 2) ? E_BAD_RATE : 0;
            break;
        }
        // Lane k records the point and a of step k, and the point the step
        // leads to.
        int pidx = 0, pa = 0, pnext = 0;
        int L = 0, a = 0;
#pragma unroll
        for (int k = 0; k < LAT_W; ++k) {
            pidx = lane == k ? L : pidx;
            pa = lane == k ? a : pa;
            const int d = (int)((P.first >> L) & 1ull);
            a += d;
            L += k + 1 + d;
            pnext = lane == k ? L : pnext;
        }
        const double tp = __shfl(P.tau, pidx, WAVE);
        const int chk_next = __shfl(P.chk, pnext < WAVE ? pnext : 0, WAVE);
        // the time chain: lane k keeps the time before step k; t + tau of
        // each step is one addition, in order
        double tl = t;
#pragma unroll
        for (int k = 0; k < LAT_W; ++k) {
            tl = lane == k ? t : tl;
            t = t + read_lane(tp, k);
        }
        // first step whose draw would cross the boundary, first step whose
        // transition leads to a state that fails its checks (the last step's
        // successor is checked by the next window), and the step whose draw
        // would exceed the step limit.  A failing state's tau of +inf can add
        // a crossing one step after the failure, which the failure precedes.
        const unsigned long long cross = __ballot(lane < LAT_W && tl + tp >= T);
        const unsigned long long fail = __ballot(lane + 1 < LAT_W && chk_next != 0);
        const int kc = cross ? __builtin_ctzll(cross) : WAVE;
        const int kf = fail ? __builtin_ctzll(fail) : WAVE;
        const int kl = near_limit ? (int)(STEP_LIMIT - g) : WAVE;
        int kend, aend;
        bool done = true;
        if (kl < LAT_W && kl <= kc && kl <= kf) {
            // the draw with index STEP_LIMIT: the implementation limit
            kend = kl;
            aend = __builtin_amdgcn_readlane(pa, kl);
            nd += (uint32_t)kl;
            ntr += (uint32_t)kl;
            rc = E_STEP_LIMIT;
        } else if (kc <= kf && kc < LAT_W) {
            // stops at the boundary before the transition of step kc
            kend = kc;
            aend = __builtin_amdgcn_readlane(pa, kc);
            nd += (uint32_t)kc + 1u;
            ntr += (uint32_t)kc;
        } else if (kf < LAT_W) {
            // the transition of step kf leads to a failing state
            kend = kf + 1;
            aend = __builtin_amdgcn_readlane(pa, kf + 1);
            const int code = __builtin_amdgcn_readlane(chk_next, kf);
            rc = (code & 1) ? E_NEG_STATE : (code & 2) ? E_BAD_RATE : 0;
            nd += (uint32_t)kf + 1u;
            ntr += (uint32_t)kf + 1u;
        } else {
            kend = LAT_W;
            aend = a;
            nd += (uint32_t)LAT_W;
            ntr += (uint32_t)LAT_W;
            done = false;
        }
#pragma unroll
        for (int c = 0; c < M::NC; ++c) s.u[c] += aend * S0[c] + (kend - aend) * S1[c];
        if (done) break;
        // the window ran through: the next one's pass
        ensure_block(g + LAT_W);
        const int src = (int)(g + LAT_W - mb) + lsrc;
        P = lattice_pass<M>(s, s.u, lk, la, S0, S1, __shfl(mine.e, src, WAVE), __shfl(mine.r2, src, WAVE));
    }
    if (lane == 0) {
        draws += nd;
        transitions += ntr;
    }
    return rc;
}

// The lattice walk for a node carried by GRP_LANES lanes (a group; a
// wavefront holds WAVE / GRP_LANES of them, each on its own node).  Lane
// (lk, la) of a group evaluates the state lk steps ahead with la transitions
// of the first kind, for the next GRP_W steps (GRP_POINTS lanes; the other
// lanes of the group idle in the pass).  The group's lanes draw GRP_BLOCK
// steps' random numbers at once (lane j draws step base + j).  Eight lanes
// and three steps a pass measured faster than sixteen and five, or four and
// two, on SIR with events over 10,000 nodes.  The path is
// read from the group's bits of one ballot; tau and the check of each point
// on it are then gathered and the steps are walked in order, each lane of
// the group doing the same (group-uniform) work, with exactly the checks and
// counts of ssa_to_boundary.  Must be called by every lane of the wavefront
// (it shuffles and ballots); `live` marks the groups whose node steps.
constexpr int GRP_LANES = GROUP_LANES;
constexpr int GRP_W = 3;
constexpr int GRP_POINTS = GRP_W * (GRP_W + 1) / 2;
constexpr int GRP_BLOCK = 6;
static_assert(GRP_POINTS < GRP_LANES && GRP_BLOCK <= GRP_LANES && GRP_BLOCK % GRP_W == 0 && WAVE % GRP_LANES == 0,
              "a group's lattice must fit its lanes");

template <class M>
__device__ __forceinline__ int ssa_group(const KParams& p, Node<M>& s, bool live, double t, double T,
                                         uint32_t day_word, uint32_t node, uint32_t stream,
                                         unsigned long long& transitions, unsigned long long& draws) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int gl = lane % GRP_LANES;
    const int gb = lane - gl;  // the group's first lane
    int lk = 0;
    while (lk < GRP_W - 1 && (lk + 1) * (lk + 2) / 2 <= gl) ++lk;
    const int la = gl < GRP_POINTS ? gl - lk * (lk + 1) / 2 : 0;
    const uint32_t k0 = (uint32_t)p.seed, k1 = (uint32_t)(p.seed >> 32);
    const uint32_t tag = stream & 0xFFFFFFu;
    int32_t S0[M::NC], S1[M::NC];
#pragma unroll
    for (int c = 0; c < M::NC; ++c) {
        S0[c] = p.S[c];
        S1[c] = p.S[c + M::NC];
    }
    uint32_t nd = 0, ntr = 0;  // group-uniform
    int rc = 0;
    bool done = !live;
    uint32_t g = 0, mb = 0;
    StepRandoms mine = step_randoms(k0, k1, (uint32_t)gl, day_word, node, tag);
    while (__any(!done)) {
        // refill the group's block when this window's draws leave it (the
        // groups still walking all sit at the same draw g)
        const bool refill = !done && g + GRP_W - mb > (uint32_t)GRP_BLOCK;
        if (__any(refill)) {
            if (refill) {
                mb = g;
                mine = step_randoms(k0, k1, g + (uint32_t)gl, day_word, node, tag);
            }
        }
        const int src = gb + (done ? 0 : (int)(g - mb)) + lk;
        const double e = __shfl(mine.e, src, WAVE);
        const double r2 = __shfl(mine.r2, src, WAVE);
        // the pass (as in lattice_pass, per group)
        int32_t uc[M::NC];
        bool neg = false;
#pragma unroll
        for (int c = 0; c < M::NC; ++c) {
            uc[c] = s.u[c] + la * S0[c] + (lk - la) * S1[c];
            neg |= uc[c] < 0;
        }
        const double c0 = M::template rate<0>(uc, s.v, s.ld, s.gd);
        const double c1 = M::template rate<1>(uc, s.v, s.ld, s.gd);
        double lam = 0.0;
        lam = lam + c0;
        lam = lam + c1;
        const double x = lam * r2;
        const int n = (c0 > 0.0 && x <= c0) ? 0 : (c1 > 0.0 ? 1 : 0);
        const int chk = neg ? 1 : !(rate_ok(c0) && rate_ok(c1)) ? 2 : !(lam > 0.0) ? 4 : 0;
        const double tau = chk ? 0.0 : e / lam;
        const unsigned long long first = __ballot(n == 0);
        const uint32_t mask = (uint32_t)(first >> gb) & ((1u << GRP_POINTS) - 1u);
        // the path: point of step k, and whether that step is of the first kind
        int pl[GRP_W], pd[GRP_W];
        int L = 0;
#pragma unroll
        for (int k = 0; k < GRP_W; ++k) {
            pl[k] = L;
            pd[k] = (int)((mask >> L) & 1u);
            L += k + 1 + pd[k];
        }
        double tk[GRP_W];
        int ck[GRP_W];
#pragma unroll
        for (int k = 0; k < GRP_W; ++k) {
            tk[k] = __shfl(tau, gb + pl[k], WAVE);
            ck[k] = __shfl(chk, gb + pl[k], WAVE);
        }
        // the steps in order: the state's checks, the step limit, the draw,
        // the day boundary, the transition
        // (as selects: the groups of a wavefront stop at different steps)
        int kapp = 0, aapp = 0;  // transitions applied in this window, of the first kind
        bool stop = done;
#pragma unroll
        for (int k = 0; k < GRP_W; ++k) {
            const bool bad = !stop && ck[k] != 0;
            const bool lim = !stop && !bad && g + (uint32_t)k == STEP_LIMIT;
            const bool draw = !stop && !bad && !lim;
            const double tn = t + tk[k];
            const bool go = draw && !(tn >= T);
            rc = bad ? ((ck[k] & 1) ? E_NEG_STATE : (ck[k] & 2) ? E_BAD_RATE : 0) : lim ? E_STEP_LIMIT : rc;
            nd += draw ? 1u : 0u;
            t = go ? tn : t;
            kapp += go ? 1 : 0;
            aapp += go ? pd[k] : 0;
            stop = stop || !go;
        }
        ntr += (uint32_t)kapp;
        if (!done) {
#pragma unroll
            for (int c = 0; c < M::NC; ++c) s.u[c] += aapp * S0[c] + (kapp - aapp) * S1[c];
            done = stop;
            g += (uint32_t)GRP_W;
        }
    }
    if (gl == 0) {
        draws += nd;
        transitions += ntr;
    }
    return rc;
}

// The select mask and shift targets of a packed event word: for the
// built-in models both are in the word (4 mask bits, 2 bits of target per
// compartment); a generated model's word holds the column of E and the
// column of N plus one (0: no shift), looked up in the model's tables.
template <class M>
__device__ __forceinline__ uint32_t event_mask(uint32_t w) {
    if constexpr (M::GENERATED)
        return M::select_mask((int)((w >> 2) & 0x3FFu));
    else
        return (w >> 2) & 0xFu;
}
template <class M>
__device__ __forceinline__ int event_target(uint32_t w, int c) {
    if constexpr (M::GENERATED) {
        const int q = (int)((w >> 12) & 0x3FFu) - 1;
        return q < 0 ? c : M::shift_target(q, c);
    } else {
        return (int)((w >> (6 + 2 * c)) & 3u);
    }
}

// One scheduled event (section 3.3) from its packed record, on node state u
// (and destination ud for an external transfer).  Indices were validated
// when the model was created.  Returns 0 or E_OVERDRAW (state unchanged).
template <class M>
__device__ __forceinline__ int apply_event(const int4 rec, const double* prop, int e, uint64_t seed,
                                           uint32_t stream, int32_t (&u)[M::NC], int32_t (&ud)[M::NC]) {
    constexpr int NC = M::NC;
    const uint32_t w = (uint32_t)rec.y;
    const int type = (int)(w & 3u);
    const uint32_t mask = event_mask<M>(w);
    // every per-compartment update below is an unconditional select so that
    // the state stays in registers (no computed addresses)
    if (type == EV_ENTER) {
        // all n individuals go to the first selected compartment
        const int first = __builtin_ctz(mask);
#pragma unroll
        for (int c = 0; c < NC; ++c) u[c] += (c == first) ? rec.z : 0;
        return 0;
    }
    int64_t total = 0;
#pragma unroll
    for (int c = 0; c < NC; ++c) total += ((mask >> c) & 1u) ? (int64_t)u[c] : 0;
    int64_t n = rec.z;
    if (n == 0) n = (int64_t)floor(prop[e] * (double)total + 0.5);
    if (n > total) return E_OVERDRAW;
    int32_t take[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) take[c] = (n == total && ((mask >> c) & 1u)) ? u[c] : 0;
    if (n < total) {
        // one individual at a time, uniformly over those not yet drawn
        EventWords words(seed, stream, (uint32_t)rec.w);
        for (int64_t k = 0; k < n; ++k) {
            const int64_t j = words.below((uint32_t)(total - k));
            int64_t below = 0;
            bool hit = false;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const bool sel = (mask >> c) & 1u;
                below += sel ? (int64_t)(u[c] - take[c]) : 0;
                const bool here = sel && !hit && j < below;
                take[c] += here ? 1 : 0;
                hit = hit || here;
            }
        }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) u[c] -= take[c];
    if (type == EV_EXIT) return 0;
    const bool ext = type == EV_EXTTRANS;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const int tgt = event_target<M>(w, c);
#pragma unroll
        for (int d = 0; d < NC; ++d) {
            const int32_t add = (tgt == d) ? take[c] : 0;
            ud[d] += ext ? add : 0;
            u[d] += ext ? 0 : add;
        }
    }
    return 0;
}

template <class M>
__device__ __forceinline__ void load_static(const KParams& p, Node<M>& s, int k, int& run) {
    run = p.node_run[k];
    const int spec = p.run_spec[run];
#pragma unroll
    for (int g = 0; g < M::NGD; ++g) s.gd[g] = p.gdata[spec * p.ngd + g];
#pragma unroll
    for (int l = 0; l < M::NLD; ++l) s.ld[l] = p.ld[(size_t)l * p.n + k];
}

// Writes the records of tspan indices [m0, m1).  All lanes of the wave call
// this together; inactive lanes contribute nothing.
template <class M>
__device__ __forceinline__ void record(const KParams& p, const Node<M>& s, int k, int run, bool active,
                                       int m0, int m1) {
    for (int m = m0; m < m1; ++m) {
        if (p.record == 0) {
            if (active) {
#pragma unroll
                for (int c = 0; c < M::NC; ++c) p.U[rec_index(m, c, k, M::NC, p.ntspan, p.n, p.nmajor)] = s.u[c];
#pragma unroll
                for (int c = 0; c < M::NV; ++c) p.V[rec_index(m, c, k, M::NV, p.ntspan, p.n, p.nmajor)] = s.v[c];
            }
        } else {
            const int lane = threadIdx.x & (WAVE - 1);
            const uint64_t act = __ballot(active);
            if (act == 0) continue;
            const int leader = __ffsll((unsigned long long)act) - 1;
            const int run0 = __shfl(run, leader, WAVE);
            const bool same = __all(!active || run == run0);
#pragma unroll
            for (int c = 0; c < M::NC; ++c) {
                const unsigned long long val = active ? (unsigned long long)(int64_t)s.u[c] : 0ull;
                if (same) {
                    const unsigned long long tot = wave_sum(val);
                    if (lane == leader)
                        atomicAdd(p.sums + ((size_t)run0 * p.ntspan + m) * p.sums_nc + c, tot);
                } else if (active) {
                    atomicAdd(p.sums + ((size_t)run * p.ntspan + m) * p.sums_nc + c, val);
                }
            }
        }
    }
}

__device__ __forceinline__ void add_counters(Ctrl* c, unsigned long long tr, unsigned long long nd,
                                             unsigned long long ev, unsigned long long dr) {
    tr = wave_sum(tr);
    nd = wave_sum(nd);
    ev = wave_sum(ev);
    dr = wave_sum(dr);
    if ((threadIdx.x & (WAVE - 1)) == 0) {
        if (tr) atomicAdd(&c->counters[0], tr);
        if (nd) atomicAdd(&c->counters[1], nd);
        if (ev) atomicAdd(&c->counters[2], ev);
        if (dr) atomicAdd(&c->counters[3], dr);
    }
}

struct Tally {
    unsigned long long tr = 0, nd = 0, ev = 0, dr = 0;
};

// The node-local event records ahead of a wavefront-wide node: lane j holds
// record from + j (the last one repeated past the node's end), so that its
// events cost one memory round trip per WAVE records rather than one each.
// Requires from < cend.
__device__ __forceinline__ int4 e1_window(const KParams& p, int from, int cend) {
    return p.e1.rec[min(from + (int)(threadIdx.x & (WAVE - 1)), cend - 1)];
}

__device__ __forceinline__ int4 read_lane4(int4 v, int lane) {
    return make_int4(__builtin_amdgcn_readlane(v.x, lane), __builtin_amdgcn_readlane(v.y, lane),
                     __builtin_amdgcn_readlane(v.z, lane), __builtin_amdgcn_readlane(v.w, lane));
}

// Loads node k's constant data and initial state (registers for the run).
// nrec: the record at cur, or, for a wavefront-wide node, the window of
// records from wbase = cur.
template <class M>
__device__ __forceinline__ void load_node(const KParams& p, int k, Node<M>& s, int& run, uint32_t& node,
                                          uint32_t& stream, int64_t& ord, int& cur, int& cend, int4& nrec,
                                          bool wide, int& wbase) {
    load_static<M>(p, s, k, run);
#pragma unroll
    for (int c = 0; c < M::NC; ++c) s.u[c] = p.u0[(size_t)c * p.n + k];
#pragma unroll
    for (int c = 0; c < M::NV; ++c) s.v[c] = p.v0[(size_t)c * p.n + k];
    node = (uint32_t)p.node_idx[k];
    stream = p.stream_base + (uint32_t)run;
    ord = p.node_ord[k];
    cur = p.e1_off[k];
    cend = p.e1_off[k + 1];
    wbase = cur;
    if (cur < cend) nrec = wide ? e1_window(p, cur, cend) : p.e1.rec[cur];
}

// The node-local events of the day (time <= T), in key order (section 3.3:
// exit, enter, internal transfer).  `counter`: the lane that counts them.
// nrec holds the record at cur, loaded ahead so that days without events
// wait for no memory access; for a wavefront-wide node (WIDE, cur and
// wbase wave-uniform) the window of records from wbase (e1_window).  A
// wide node's cursor, stream and state are the same in every lane; read
// from the first lane they are known to be uniform, so that the loop's
// control and the sampling's integer work run on the scalar unit.
template <class M, bool WIDE>
__device__ __forceinline__ void day_events(const KParams& p, Node<M>& s, int b, double T, uint32_t stream, int& cur,
                                           int cend, int4& nrec, int& wbase, bool& dead, Tally& t, bool counter) {
    if constexpr (WIDE) {
        cur = __builtin_amdgcn_readfirstlane(cur);
        cend = __builtin_amdgcn_readfirstlane(cend);
        wbase = __builtin_amdgcn_readfirstlane(wbase);
        stream = __builtin_amdgcn_readfirstlane(stream);
#pragma unroll
        for (int c = 0; c < M::NC; ++c) s.u[c] = __builtin_amdgcn_readfirstlane(s.u[c]);
    }
    while (cur < cend) {
        const int4 rec = WIDE ? read_lane4(nrec, cur - wbase) : nrec;
        if (!((double)rec.x <= T)) break;
        const int rc = apply_event<M>(rec, p.e1.prop, cur, p.seed, stream, s.u, s.u);
        if (rc) {
            raise_error(p.ctrl, b, PH_E1, p.e1.ordinal[cur], rc);
            dead = true;
            return;
        }
        t.ev += counter ? 1 : 0;
        ++cur;
        if (cur < cend) {
            if constexpr (!WIDE) {
                nrec = p.e1.rec[cur];
            } else if (cur - wbase >= WAVE) {
                wbase = cur;
                nrec = e1_window(p, cur, cend);
            }
        }
    }
}

// A day of a node carried by a group of lanes: the SSA (called by every
// lane of the wavefront) and then the day's node-local events.
template <class M>
__device__ __forceinline__ void group_day(const KParams& p, Node<M>& s, bool live, int b, int64_t day, uint32_t node,
                                          uint32_t stream, int64_t ord, int& cur, int cend, int4& nrec, bool& dead,
                                          Tally& t, bool counter) {
    const double T = (double)day;
    const double t0 = b == 0 ? p.t0 : T - 1.0;
    int rc = 0;
    if constexpr (!M::GENERATED) rc = ssa_group<M>(p, s, live, t0, T, (uint32_t)(int32_t)day, node, stream, t.tr, t.dr);
    if (!live) return;
    if (rc) {
        raise_error(p.ctrl, b, PH_SSA, ord, rc);
        dead = true;
        return;
    }
    int wbase = cur;
    day_events<M, false>(p, s, b, T, stream, cur, cend, nrec, wbase, dead, t, counter);
}

// ---------------------------------------------------------------------------
// the all events method (section 3.4, 'aem')
// ---------------------------------------------------------------------------
// Every transition channel j of a node fires when its integrated rate T_j
// reaches P_j, the running sum of unit exponentials from the channel's own
// stream (Philox block (k, j, node, stream | 2 << 24), the k-th exponential
// from the block's first two words).  The state per node and channel
// carries over from day to day; the direct method needs none.
template <class M, bool ON>
struct AemState {};
template <class M>
struct AemState<M, true> {
    double T[M::NT], P[M::NT];
    uint32_t K[M::NT];
};

__device__ __forceinline__ double aem_exp(uint64_t seed, uint32_t k, uint32_t j, uint32_t node, uint32_t stream) {
    const Block4 r = philox10((uint32_t)seed, (uint32_t)(seed >> 32), k, j, node, (stream & 0xFFFFFFu) | (2u << 24));
    return -series_log(open_uniform(r.x, r.y));
}

template <class M>
__device__ __forceinline__ double rate_at(int j, const Node<M>& s) {
    if constexpr (M::GENERATED)
        return M::rate(j, s.u, s.v, s.ld, s.gd);
    else
        return j == 0 ? M::template rate<0>(s.u, s.v, s.ld, s.gd) : M::template rate<1>(s.u, s.v, s.ld, s.gd);
}

template <class M>
__device__ __forceinline__ void aem_load(const KParams& p, int k, AemState<M, true>& a) {
#pragma unroll
    for (int j = 0; j < M::NT; ++j) {
        a.T[j] = p.aem_T[(size_t)j * p.n + k];
        a.P[j] = p.aem_P[(size_t)j * p.n + k];
        a.K[j] = p.aem_K[(size_t)j * p.n + k];
    }
}

template <class M>
__device__ __forceinline__ void aem_store(const KParams& p, int k, const AemState<M, true>& a) {
#pragma unroll
    for (int j = 0; j < M::NT; ++j) {
        p.aem_T[(size_t)j * p.n + k] = a.T[j];
        p.aem_P[(size_t)j * p.n + k] = a.P[j];
        p.aem_K[(size_t)j * p.n + k] = a.K[j];
    }
}

// One node from t to the day boundary T: the channel with the least
// (P_j - T_j)/w_j fires (the lowest j on a tie) unless that time crosses T;
// the other channels' integrals advance by w tau, the fired one's becomes
// P_j and P_j takes the channel's next exponential; at the boundary every
// integral advances by w (T - t).  The same checks as the direct method:
// the step limit before each step, a negative compartment after a
// transition, bad rates.  Channel arrays are indexed through unrolled
// selects, so they stay in registers.
template <class M>
__device__ __forceinline__ int ssa_aem(const KParams& p, Node<M>& s, AemState<M, true>& a, double t, double T,
                                       uint32_t node, uint32_t stream, unsigned long long& transitions,
                                       unsigned long long& draws) {
    double w[M::NT];
    bool bad = false;
#pragma unroll
    for (int j = 0; j < M::NT; ++j) {
        w[j] = rate_at<M>(j, s);
        bad = bad || !rate_ok(w[j]);
    }
    if (bad) return E_BAD_RATE;
    for (uint32_t k = 0;; ++k) {
        int n = -1;
        double best = 0.0;
#pragma unroll
        for (int j = 0; j < M::NT; ++j) {
            const double tau = (a.P[j] - a.T[j]) / w[j];
            const bool take = w[j] > 0.0 && (n < 0 || tau < best);
            best = take ? tau : best;
            n = take ? j : n;
        }
        if (n < 0) return 0;
        if (k == STEP_LIMIT) return E_STEP_LIMIT;
        draws += 1;
        const double tn = t + best;
        if (tn >= T) {
            const double rest = T - t;
#pragma unroll
            for (int j = 0; j < M::NT; ++j) a.T[j] = a.T[j] + w[j] * rest;
            return 0;
        }
        double pn = 0.0;
        uint32_t kn = 0;
#pragma unroll
        for (int j = 0; j < M::NT; ++j) {
            pn = j == n ? a.P[j] : pn;
            kn = j == n ? a.K[j] : kn;
        }
        const double pnext = pn + aem_exp(p.seed, kn, (uint32_t)n, node, stream);
#pragma unroll
        for (int j = 0; j < M::NT; ++j) {
            const bool f = j == n;
            a.T[j] = f ? a.P[j] : a.T[j] + w[j] * best;
            a.P[j] = f ? pnext : a.P[j];
            a.K[j] = f ? a.K[j] + 1u : a.K[j];
        }
        t = tn;
        uint32_t g;
        if constexpr (M::GENERATED) {
            M::apply(n, s.u);
            g = M::deps(n);
        } else {
#pragma unroll
            for (int c = 0; c < M::NC; ++c) s.u[c] += n ? p.S[c + M::NC] : p.S[c];
            g = n ? p.Gmask[1] : p.Gmask[0];
        }
        transitions += 1;
        bool neg = false;
#pragma unroll
        for (int c = 0; c < M::NC; ++c) neg = neg || s.u[c] < 0;
        if (neg) return E_NEG_STATE;
#pragma unroll
        for (int j = 0; j < M::NT; ++j)
            if ((g >> j) & 1u) {
                w[j] = rate_at<M>(j, s);
                bad = bad || !rate_ok(w[j]);
            }
        if (bad) return E_BAD_RATE;
    }
}

// SSA to day boundary b, then the node's E1 events with time <= T.  With
// wide, the whole wavefront carries the node (the lattice walk, or the plain
// chain when G does not mark both rates); event tallies are then kept by
// lane 0 only.  With AEM, the all events method on one lane.
template <class M, bool PIPE, bool AEM = false>
__device__ __forceinline__ void ssa_and_e1(const KParams& p, Node<M>& s, int b, int64_t day, uint32_t node,
                                           uint32_t stream, int64_t ord, int& cur, int cend, int4& nrec, int& wbase,
                                           bool& dead, Tally& t, bool wide, AemState<M, AEM>& a) {
    const double T = (double)day;
    const double t0 = b == 0 ? p.t0 : T - 1.0;
    const uint32_t dw = (uint32_t)(int32_t)day;
    int rc = 0;
    if constexpr (AEM)
        rc = ssa_aem<M>(p, s, a, t0, T, node, stream, t.tr, t.dr);
    else if constexpr (M::GENERATED)
        rc = ssa_to_boundary<M, PIPE>(p, s, t0, T, dw, node, stream, t.tr, t.dr);  // never wide
    else
        rc = !wide       ? ssa_to_boundary<M, PIPE>(p, s, t0, T, dw, node, stream, t.tr, t.dr)
             : p.lattice ? ssa_lattice<M>(p, s, t0, T, dw, node, stream, t.tr, t.dr)
                         : ssa_wide<M>(p, s, t0, T, dw, node, stream, t.tr, t.dr);
    if (rc) {
        raise_error(p.ctrl, b, PH_SSA, ord, rc);
        dead = true;
        return;
    }
    // (the branch is uniform: a wavefront carries one wide node or none)
    if (wide)
        day_events<M, true>(p, s, b, T, stream, cur, cend, nrec, wbase, dead, t, (threadIdx.x & (WAVE - 1)) == 0);
    else
        day_events<M, false>(p, s, b, T, stream, cur, cend, nrec, wbase, dead, t, true);
}

// ---------------------------------------------------------------------------
// free-running kernel (no external transfers)
// ---------------------------------------------------------------------------
template <class M, bool PIPE, bool GRP, bool AEM = false>
__global__ void __launch_bounds__(256) free_kernel(KParams pa) {
    KParams p = pa;
    p.seed = pa.rp->seed;
    p.stream_base = pa.rp->stream_base;
    const int lane = threadIdx.x & (WAVE - 1);
    Tally t;
    for (;;) {
        unsigned chunk = 0;
        if (lane == 0) chunk = atomicAdd(&p.ctrl->work[p.group], 1u);
        chunk = __shfl(chunk, 0, WAVE);
        if (chunk >= (unsigned)p.nchunks) break;
        // chunks [0, nbig): one heavy node per wavefront; then ngw chunks of
        // WAVE / GRP_LANES nodes with GRP_LANES lanes each; then pack nodes per chunk
        const int c = (int)chunk;
        const bool wide = c < p.nbig;
        const bool grp = GRP && !wide && c < p.nbig + p.ngw;
        const int k = wide  ? c
                      : grp ? p.nbig + (c - p.nbig) * (WAVE / GRP_LANES) + lane / GRP_LANES
                            : p.nbig + p.ngrp + (c - p.nbig - p.ngw) * p.pack + lane;
        const bool active = (wide || (grp ? k < p.nbig + p.ngrp : lane < p.pack)) && k < p.n;
        const bool owner = active && (wide ? lane == 0 : grp ? lane % GRP_LANES == 0 : true);  // writes records
        Node<M> s{};
        int run = 0, cur = 0, cend = 0;
        uint32_t node = 0, stream = 0;
        int64_t ord = 0;
        int4 nrec = make_int4(0, 0, 0, 0);
        int wbase = 0;
        AemState<M, AEM> a{};
        if (active) {
            load_node<M>(p, k, s, run, node, stream, ord, cur, cend, nrec, wide, wbase);
            if constexpr (AEM) aem_load<M>(p, k, a);
        }

        bool dead = false;
        uint64_t key_raw = 0;  // error key, refreshed every 8 days and read 8 days later
        for (int b = 0; b < p.nb; ++b) {
            if ((b & 7) == 0) {
                if (b > 0 && (__shfl(key_raw, 0, WAVE) >> 44) < (uint64_t)b) break;
                if (lane == 0)
                    key_raw = __hip_atomic_load(&p.ctrl->err_key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            const int64_t day = p.T1 + b;
            if (grp) group_day<M>(p, s, active && !dead, b, day, node, stream, ord, cur, cend, nrec, dead, t, owner);
            if (active && !dead) {
                if (!grp)
                    ssa_and_e1<M, PIPE, AEM>(p, s, b, day, node, stream, ord, cur, cend, nrec, wbase, dead, t, wide, a);
                if (!dead && !M::pts(s.v, s.u, s.ld, s.gd, day)) {
                    if (owner) raise_error(p.ctrl, b, PH_PTS, ord, E_PTS);
                    dead = true;
                }
                t.nd += owner ? 1 : 0;
            }
            record<M>(p, s, k, run, owner, p.rec_off[b], p.rec_off[b + 1]);
        }
    }
    add_counters(p.ctrl, t.tr, t.nd, t.ev, t.dr);
}

// ---------------------------------------------------------------------------
// lane-queue kernel (no external transfers, one lane per node, lanes advance
// independently)
// ---------------------------------------------------------------------------
// In free_kernel a wavefront's nodes go through each day together, so a day
// costs the wavefront as many steps as its busiest node needs that day, and
// a node whose epidemic has died out keeps its lane to the end.  Here every
// lane advances its own node: an iteration draws one step for each lane
// that is inside a day, and a lane whose step crosses its day boundary (or
// whose day has no positive rate) closes that day -- node-local events,
// post-time step, records -- and opens the next one.  A lane whose node has
// finished its last day takes the next node of its wavefront's chunk
// (consecutive nodes of one run, heaviest first); the wavefront takes a new
// chunk from the work queue when its chunk has been handed out.  A node
// that can no longer change (every rate zero, no event left, a state the
// post-time step maps to itself) is finished at once: its state is recorded
// for every remaining tspan point.  Per-run sums are accumulated per chunk
// in LDS (a wavefront holds at most LQ_SLOTS chunks) and added to the global
// sums when the chunk's last node is done.  Each node goes through exactly
// the operations of ssa_to_boundary and day_events, so every result is
// bit-identical to the other kernels'.
// Per-lane state of the lane-queue kernel.  The run's global data sit in the
// lane's LDS slot, and the counters in LDS per wavefront, to leave the
// registers to the SSA.
template <class M>
struct LaneState {
    int32_t u[M::NC];
    double v[M::NV > 0 ? M::NV : 1];
    double ld[M::NLD > 0 ? M::NLD : 1];
    int k = -1;  // node, -1 when the lane is free
    int slot = 0, b = 0, cur = 0, cend = 0;
    int etime = 0;      // time of the node's next node-local event
    bool open = false;  // inside a day with lambda > 0: the next draw is due
    uint32_t node = 0, tag = 0, step = 0;
    uint32_t dd = 0, dt = 0;  // draws and transitions of the current day
    int fail = 0;             // an error of the current day's SSA (code), taken up at its end
    double e = 0.0, r2 = 0.0; // with pipelining: the random numbers of the next draw
    double t = 0.0, T = 0.0, w0 = 0.0, w1 = 0.0, lam = 0.0;
};

// Counters of a wavefront in LDS: transitions, node-days, events, draws.
enum { LQ_TR = 0, LQ_ND = 1, LQ_EV = 2, LQ_DR = 3, LQ_TALLIES = 4 };

// Records the state at the tspan indices [m0, m1): into the lane's LDS slot
// (sums) or the trajectory buffer.
template <class M>
__device__ __forceinline__ void lane_record(const KParams& p, const LaneState<M>& L, unsigned long long* slotbase,
                                            int m0, int m1) {
    for (int m = m0; m < m1; ++m) {
        if (p.record != 0) {
#pragma unroll
            for (int c = 0; c < M::NC; ++c)
                atomicAdd(slotbase + m * M::NC + c, (unsigned long long)(int64_t)L.u[c]);
        } else {
#pragma unroll
            for (int c = 0; c < M::NC; ++c) p.U[rec_index(m, c, L.k, M::NC, p.ntspan, p.n, 0)] = L.u[c];
#pragma unroll
            for (int c = 0; c < M::NV; ++c) p.V[rec_index(m, c, L.k, M::NV, p.ntspan, p.n, 0)] = L.v[c];
        }
    }
}

// Ends the lane's node after an error of `phase` at its current day.
template <class M>
__device__ __forceinline__ void lane_fail(const KParams& p, LaneState<M>& L, int phase, int64_t ord, int code,
                                          unsigned long long* tally) {
    raise_error(p.ctrl, L.b, phase, ord, code);
    atomicAdd(tally + LQ_DR, (unsigned long long)L.dd);
    atomicAdd(tally + LQ_TR, (unsigned long long)L.dt);
    atomicAdd(tally + LQ_ND, 1ull);
    L.k = -1;
    L.open = false;
}

// Opens day b of the lane's node: all rates from the state (Appendix A, a
// new unit of time), lambda, and whether a draw is due.  A node whose rates
// are all zero with no event left and a fixed point of the post-time step
// is finished here, its state recorded for the rest of the run.
template <class M, bool PIPE>
__device__ __forceinline__ void lane_open_day(const KParams& p, LaneState<M>& L, unsigned long long* slotbase,
                                              const double* gd, const int* rec_off, unsigned long long* tally) {
    L.T = (double)(p.T1 + L.b);
    L.t = L.b == 0 ? p.t0 : L.T - 1.0;
    L.step = 0;
    L.fail = 0;
    L.dd = 0;
    L.dt = 0;
    L.w0 = M::template rate<0>(L.u, L.v, L.ld, gd);
    L.w1 = M::template rate<1>(L.u, L.v, L.ld, gd);
    if (!rate_ok(L.w0) || !rate_ok(L.w1)) {
        lane_fail<M>(p, L, PH_SSA, p.node_ord[L.k], E_BAD_RATE, tally);
        return;
    }
    double lam = 0.0;
    lam = lam + L.w0;
    lam = lam + L.w1;
    L.lam = lam;
    L.open = lam > 0.0;
    if (PIPE && L.open) {
        const StepRandoms r = step_randoms((uint32_t)p.rp->seed, (uint32_t)(p.rp->seed >> 32), 0u,
                                           (uint32_t)(int32_t)(p.T1 + L.b), L.node, L.tag);
        L.e = r.e;
        L.r2 = r.r2;
    }
    if (!L.open && L.cur >= L.cend && M::pts_fixed(L.v, L.u)) {
        lane_record<M>(p, L, slotbase, rec_off[L.b], p.ntspan);
        atomicAdd(tally + LQ_ND, (unsigned long long)(p.nb - L.b));
        L.k = -1;
    }
}

// Loads node k (of the run `run`) into a free lane.
template <class M>
__device__ __forceinline__ void lane_load(const KParams& p, LaneState<M>& L, int k, int slot, int run,
                                          uint32_t stream_base) {
    L.k = k;
    L.slot = slot;
#pragma unroll
    for (int c = 0; c < M::NC; ++c) L.u[c] = p.u0[(size_t)c * p.n + k];
#pragma unroll
    for (int c = 0; c < M::NV; ++c) L.v[c] = p.v0[(size_t)c * p.n + k];
#pragma unroll
    for (int l = 0; l < M::NLD; ++l) L.ld[l] = p.ld[(size_t)l * p.n + k];
    L.node = (uint32_t)p.node_idx[k];
    L.tag = (stream_base + (uint32_t)run) & 0xFFFFFFu;
    L.cur = p.e1_off[k];
    L.cend = p.e1_off[k + 1];
    L.etime = L.cur < L.cend ? p.e1.rec[L.cur].x : 0;
    L.b = 0;
}

template <class M, bool PIPE>
__global__ void __launch_bounds__(256) lane_kernel(KParams pa) {
    extern __shared__ unsigned long long lq_lds[];
    const KParams& p = pa;
    const uint64_t seed = p.rp->seed;
    const uint32_t stream_base = p.rp->stream_base;
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const int lane = threadIdx.x & (WAVE - 1);
    const unsigned long long lt_mask = (1ull << lane) - 1ull;
    const bool sums = p.record != 0;
    const int per_slot = sums ? p.ntspan * M::NC : 0;
    // LDS: the tspan indices recorded after each day (read at every day's
    // end), then per wavefront its recording slots, its slots' global data
    // and its counters
    int* rec_off = (int*)lq_lds;
    for (int i = threadIdx.x; i <= p.nb; i += blockDim.x) rec_off[i] = p.rec_off[i];
    const int per_wave = LQ_SLOTS * per_slot + LQ_SLOTS * M::NGD + LQ_TALLIES;
    unsigned long long* mine = lq_lds + (p.nb + 2) / 2 + (size_t)(threadIdx.x / WAVE) * per_wave;
    double* gdl = (double*)(mine + LQ_SLOTS * per_slot);
    unsigned long long* tally = mine + LQ_SLOTS * per_slot + LQ_SLOTS * M::NGD;
    for (int i = lane; i < per_wave; i += WAVE) mine[i] = 0ull;
    __syncthreads();
    // wavefront-uniform: the run of each slot (-1 free), the chunk being handed out
    int srun0 = -1, srun1 = -1;
    int cslot = -1, next = 0, stop = 0;
    bool drained = false;
    LaneState<M> L;
    // adds a slot's sums to the global ones and clears it
    auto flush = [&](int sl, int r) {
        unsigned long long* base = mine + sl * per_slot;
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        for (int i = lane; i < per_slot; i += WAVE) {
            const unsigned long long v = base[i];
            if (v) atomicAdd(p.sums + ((size_t)r * p.ntspan + i / M::NC) * p.sums_nc + i % M::NC, v);
            base[i] = 0ull;
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
    };
    for (unsigned round = 0;; ++round) {
        // the first error's day: nodes past it stop (their later records are
        // undefined); refreshed every 8 rounds
        if ((round & 7u) == 0) {
            uint64_t key = 0;
            if (lane == 0) key = __hip_atomic_load(&p.ctrl->err_key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint64_t err_day = __shfl(key, 0, WAVE) >> 44;
            if (L.k >= 0 && (uint64_t)L.b > err_day) {
                L.k = -1;
                L.open = false;
            }
        }
        // ---- free lanes: finished chunks are flushed, new nodes handed out
        unsigned long long freem = __ballot(L.k < 0);
        if (freem) {
            if (srun0 >= 0 && !(cslot == 0 && next < stop) && !__ballot(L.k >= 0 && L.slot == 0)) {
                if (sums) flush(0, srun0);
                srun0 = -1;
                if (cslot == 0) cslot = -1;
            }
            if (srun1 >= 0 && !(cslot == 1 && next < stop) && !__ballot(L.k >= 0 && L.slot == 1)) {
                if (sums) flush(1, srun1);
                srun1 = -1;
                if (cslot == 1) cslot = -1;
            }
            while (freem) {
                if (cslot < 0 || next >= stop) {
                    const int fs = srun0 < 0 ? 0 : srun1 < 0 ? 1 : -1;
                    if (drained || fs < 0) break;
                    unsigned c = 0;
                    if (lane == 0) c = atomicAdd(&p.ctrl->work[p.group], 1u);
                    c = __shfl(c, 0, WAVE);
                    if (c >= (unsigned)p.nlchunks) {
                        drained = true;
                        break;
                    }
                    const int4 ch = p.lchunks[c];
                    cslot = fs;
                    if (fs == 0)
                        srun0 = ch.z;
                    else
                        srun1 = ch.z;
                    next = ch.x;
                    stop = ch.y;
                    // the run's global data into the slot (the slot is free:
                    // no lane reads it)
                    if (lane < M::NGD) gdl[fs * M::NGD + lane] = p.gdata[(size_t)p.run_spec[ch.z] * p.ngd + lane];
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                }
                const int take = min(__popcll(freem), stop - next);
                const int rank = __popcll(freem & lt_mask);
                const bool me = ((freem >> lane) & 1ull) && rank < take;
                if (me) {
                    lane_load<M>(p, L, next + rank, cslot, cslot == 0 ? srun0 : srun1, stream_base);
                    lane_open_day<M, PIPE>(p, L, mine + L.slot * per_slot, gdl + L.slot * M::NGD, rec_off, tally);
                }
                next += take;
                freem &= ~__ballot(me);
            }
        }
        if (!__ballot(L.k >= 0)) {
            if (drained) break;
            continue;
        }
        // ---- draws: one step of ssa_to_boundary's loop for every lane inside
        // a day, until lq_batch lanes wait at the end of a day or have no node
        // (or no lane has a draw due); those are then served together
        for (;;) {
            if (L.open) {
                // the step limit, the draw, the day boundary and the
                // transition as selects (one branch for the whole step); an
                // error is taken up with the lane's day end
                const bool lim = L.step == STEP_LIMIT;
                const uint32_t dw = (uint32_t)(int32_t)(p.T1 + L.b);
                // with PIPE the step's numbers were computed by the previous
                // step, which computes the next step's (kept only if the day
                // goes on) beside its own dependent chain
                StepRandoms r, rn{0.0, 0.0};
                if constexpr (PIPE) {
                    r = {L.e, L.r2};
                    rn = step_randoms(k0, k1, L.step + 1u, dw, L.node, L.tag);
                } else {
                    r = step_randoms(k0, k1, L.step, dw, L.node, L.tag);
                }
                const double tau = r.e / L.lam;
                const double tn = L.t + tau;
                const Transition<M> nx =
                    transition_of<M>(p, L.u, L.v, L.ld, gdl + L.slot * M::NGD, L.w0, L.w1, L.lam * r.r2);
                const bool go = !lim && !(tn >= L.T);
                L.dd += lim ? 0u : 1u;
                L.dt += go ? 1u : 0u;
                L.t = go ? tn : L.t;
#pragma unroll
                for (int c = 0; c < M::NC; ++c) L.u[c] = go ? nx.u[c] : L.u[c];
                L.w0 = go ? nx.w0 : L.w0;
                L.w1 = go ? nx.w1 : L.w1;
                double lam = 0.0;
                lam = lam + L.w0;
                lam = lam + L.w1;
                L.lam = lam;
                L.fail = lim ? E_STEP_LIMIT : go ? nx.err : 0;
                L.open = go && nx.err == 0 && lam > 0.0;
                L.step += L.open ? 1u : 0u;
                if constexpr (PIPE) {
                    L.e = rn.e;
                    L.r2 = rn.r2;
                }
            }
            const unsigned long long idle = __ballot(!L.open);
            if (__popcll(idle) >= (unsigned)p.lq_batch || idle == ~0ull) break;
        }
        // ---- day end: node-local events, post-time step, records, next day
        if (L.k >= 0 && !L.open) {
            const double* gd = gdl + L.slot * M::NGD;
            unsigned long long* slotbase = mine + L.slot * per_slot;
            atomicAdd(tally + LQ_DR, (unsigned long long)L.dd);
            atomicAdd(tally + LQ_TR, (unsigned long long)L.dt);
            L.dd = 0;
            L.dt = 0;
            bool dead = L.fail != 0;
            if (dead) lane_fail<M>(p, L, PH_SSA, p.node_ord[L.k], L.fail, tally);
            while (!dead && L.cur < L.cend && (double)L.etime <= L.T) {
                const int rc = apply_event<M>(p.e1.rec[L.cur], p.e1.prop, L.cur, seed, L.tag, L.u, L.u);
                if (rc) {
                    lane_fail<M>(p, L, PH_E1, p.e1.ordinal[L.cur], rc, tally);
                    dead = true;
                    break;
                }
                atomicAdd(tally + LQ_EV, 1ull);
                ++L.cur;
                if (L.cur < L.cend) L.etime = p.e1.rec[L.cur].x;
            }
            if (!dead && !M::pts(L.v, L.u, L.ld, gd, p.T1 + L.b)) {
                lane_fail<M>(p, L, PH_PTS, p.node_ord[L.k], E_PTS, tally);
                dead = true;
            }
            if (!dead) {
                atomicAdd(tally + LQ_ND, 1ull);
                lane_record<M>(p, L, slotbase, rec_off[L.b], rec_off[L.b + 1]);
                L.b += 1;
                if (L.b >= p.nb)
                    L.k = -1;
                else
                    lane_open_day<M, PIPE>(p, L, slotbase, gd, rec_off, tally);
            }
        }
    }
    // nodes finished at once in the last hand-out may have left records in a slot
    if (sums) {
        if (srun0 >= 0) flush(0, srun0);
        if (srun1 >= 0) flush(1, srun1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (lane == 0) {
        for (int i = 0; i < LQ_TALLIES; ++i) {
            const unsigned long long v = tally[i];
            if (v) atomicAdd(&p.ctrl->counters[i == LQ_TR ? 0 : i == LQ_ND ? 1 : i == LQ_EV ? 2 : 3], v);
        }
    }
}

// ---------------------------------------------------------------------------
// dataflow kernel (external transfers, every node resident)
// ---------------------------------------------------------------------------
constexpr unsigned long long MAIL_PACKED = 1ull << 63;  // counts packed in bits 0..47
constexpr unsigned long long MAIL_SIDE = 1ull << 62;    // counts in mail_big (release/acquire)

// Posts the counts a transfer delivers: up to three 16-bit counts in one
// atomic word, else through the side array.
template <int NC>
__device__ __forceinline__ void post_mail(const KParams& p, int e, const int32_t (&cnt)[NC]) {
    bool small = true;
#pragma unroll
    for (int c = 0; c < NC; ++c) small = small && cnt[c] <= 0xFFFF;
    if (small && NC <= 3) {
        unsigned long long w = MAIL_PACKED;
#pragma unroll
        for (int c = 0; c < NC; ++c) w |= (unsigned long long)cnt[c] << (16 * c);
        __hip_atomic_store(&p.mail[e], w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
#pragma unroll
        for (int c = 0; c < NC; ++c) p.mail_big[(size_t)e * NC + c] = cnt[c];
        __hip_atomic_store(&p.mail[e], MAIL_SIDE, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Adds the counts of a posted mailbox word w to u.
template <int NC>
__device__ __forceinline__ void take_mail(const KParams& p, int e, unsigned long long w, int32_t (&u)[NC]) {
    if (w & MAIL_PACKED) {
#pragma unroll
        for (int c = 0; c < NC; ++c) u[c] += (int32_t)((w >> (16 * c)) & 0xFFFFull);
    } else {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
#pragma unroll
        for (int c = 0; c < NC; ++c) u[c] += p.mail_big[(size_t)e * NC + c];
    }
}

// The coupling sum of a spatially coupled post-time step (SISe_sp): every
// node posts its continuous state before the step and its size after the
// day's events, waits for the day's posts of its neighbours, then adds up
// their coupling terms in stored order.  Every node posts before it waits,
// so every wait ends (all node wavefronts are resident in this kernel).
// Posts alternate between two buffers by day parity.  A node also waits for
// the day's posts of the nodes that read it (whether or not it reads them,
// and whatever its size): it can then overwrite a buffer two days on only
// after every reader has posted the next day, that is, has finished reading
// the post it overwrites.  The wait looks at CPL_PEEK posts at once, so that
// their round trips to memory overlap; one acquire fence then covers every
// post read.
// Called by every lane of the wavefront (the wait loop is wave-uniform);
// `active` lanes carry a node, `owner` is the lane that posts for it, and
// nodes that an error stopped keep posting their last state.  c is 0 for an
// empty node.  A wait longer than the wall-clock limit abandons the run; an
// earlier error lets the waits give up (the run's later results are
// undefined).
constexpr int CPL_PEEK = 8;

template <class M>
__device__ __forceinline__ double coupled_sum(const KParams& p, const Node<M>& s, int k, int b, bool active,
                                              bool owner) {
    const int32_t ni = s.u[0] + s.u[1];
    CplPost* post = p.cpl_post + (size_t)(b & 1) * p.n;
    if (owner) {
        post[k].phi = s.v[0];
        post[k].n = ni;
        __hip_atomic_store(&post[k].day, b, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
    const int e0 = active ? p.cpl_off[k] : 0;
    const int eend = active ? p.cpl_off[k + 1] : 0;
    int e = e0;
    unsigned spins = 0;
    WaitClock clock;
    while (__any(e < eend)) {
        int32_t d[CPL_PEEK];
#pragma unroll
        for (int q = 0; q < CPL_PEEK; ++q)
            d[q] = e + q < eend
                       ? __hip_atomic_load(&post[p.cpl_idx[e + q]].day, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                       : b;
        int ready = 0;
        bool gap = false;
#pragma unroll
        for (int q = 0; q < CPL_PEEK; ++q) {
            gap = gap || d[q] != b;
            ready += gap ? 0 : 1;
        }
        e = min(e + ready, eend);
        if (!__any(ready > 0) && (++spins & 255u) == 0) {
            const bool quit = __hip_atomic_load(&p.ctrl->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ||
                              load_error_step(p.ctrl) < (uint64_t)b;
            const bool late = __shfl(clock.expired(p.wait_ticks) ? 1 : 0, 0, WAVE) != 0;
            if (late && (threadIdx.x & (WAVE - 1)) == 0)
                __hip_atomic_store(&p.ctrl->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (__any(quit) || late) break;
            __builtin_amdgcn_s_sleep(1);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    double c = 0.0;
    if (active && ni > 0) {
        const int fend = p.cpl_fend[k];
#pragma unroll 4
        for (int f = e0; f < fend; ++f) {
            const int j = p.cpl_idx[f];
            c = c + M::coupling_term(post[j].phi, post[j].n, s.v[0], ni, p.cpl_w[f]);
        }
    }
    return c;
}

template <class M, bool PIPE, bool GRP, bool AEM = false>
__global__ void __launch_bounds__(256) flow_kernel(KParams pa) {
    KParams p = pa;
    p.seed = pa.rp->seed;
    p.stream_base = pa.rp->stream_base;
    Tally t;
    const int lane = threadIdx.x & (WAVE - 1);
    const int wpb = blockDim.x / WAVE;
    const int line_g = 32 / (p.pack * wpb);  // workgroups whose records fill one 128-byte line
    const int gw = xcd_block(blockIdx.x, (p.nbig + p.ngw + wpb - 1) / wpb, gridDim.x, line_g) * wpb +
                   (int)(threadIdx.x / WAVE);
    // waves [0, nbig): one heavy node per wavefront
    const bool wide = gw < p.nbig;
    // then ngw waves of WAVE / GRP_LANES nodes with GRP_LANES lanes each
    const bool grp = GRP && !wide && gw < p.nbig + p.ngw;
    // then pack nodes per wave, one lane each
    const int k = wide  ? gw
                  : grp ? p.nbig + (gw - p.nbig) * (WAVE / GRP_LANES) + lane / GRP_LANES
                        : p.nbig + p.ngrp + (gw - p.nbig - p.ngw) * p.pack + lane;
    const bool active = (wide || (grp ? k < p.nbig + p.ngrp : lane < p.pack)) && k < p.n;
    const bool owner = active && (wide ? lane == 0 : grp ? lane % GRP_LANES == 0 : true);
    Node<M> s{};
    int run = 0, cur = 0, cend = 0, tcur = 0, tend = 0;
    uint32_t node = 0, stream = 0;
    int64_t ord = 0;
    int4 nrec = make_int4(0, 0, 0, 0), item = make_int4(0, NO_STEP, 0, 0), trec = make_int4(0, 0, 0, 0);
    int wbase = 0;
    AemState<M, AEM> a{};
    if (active) {
        load_node<M>(p, k, s, run, node, stream, ord, cur, cend, nrec, wide, wbase);
        if constexpr (AEM) aem_load<M>(p, k, a);
        tcur = p.e2n_off[k];
        tend = p.e2n_off[k + 1];
        if (tcur < tend) {
            item = p.e2n_item[tcur];
            trec = p.e2n_rec[tcur];
        }

    }
    bool dead = false;
    uint64_t key_raw = 0;  // error key, refreshed every 8 days and read 8 days later
    for (int b = 0; b < p.nb; ++b) {
        if ((b & 7) == 0) {
            if (b > 0 && (__shfl(key_raw, 0, WAVE) >> 44) < (uint64_t)b) break;
            if (lane == 0)
                key_raw = __hip_atomic_load(&p.ctrl->err_key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        const int64_t day = p.T1 + b;
        if (grp)
            group_day<M>(p, s, active && !dead, b, day, node, stream, ord, cur, cend, nrec, dead, t, owner);
        else if (active && !dead)
            ssa_and_e1<M, PIPE, AEM>(p, s, b, day, node, stream, ord, cur, cend, nrec, wbase, dead, t, wide, a);

        // this step's external transfers of the node, in key order.  The loop
        // is uniform over the wavefront and every lane that can move on does:
        // sources never wait, so no lane can block another one of its wave.
        bool pending = active && item.y == b;
        unsigned spins = 0;
        WaitClock clock;
        while (__any(pending)) {
            bool moved = false;
            if (pending) {
                const int e = item.x;
                if (item.z != 1) {
                    // source (or source and destination): sample and post
                    int32_t got[M::NC];
#pragma unroll
                    for (int c = 0; c < M::NC; ++c) got[c] = 0;
                    const uint32_t ev_stream = p.stream_base + (uint32_t)item.w;
                    int rc = dead ? 0 : apply_event<M>(trec, p.e2.prop, e, p.seed, ev_stream, s.u, got);
                    if (rc) {
                        if (owner) raise_error(p.ctrl, b, PH_E2, p.e2.ordinal[e], rc);
                        dead = true;
                    }
                    if (item.z == 2) {
#pragma unroll
                        for (int c = 0; c < M::NC; ++c) s.u[c] += got[c];
                    } else if (owner) {
                        post_mail<M::NC>(p, e, got);
                    }
                    t.ev += (owner && !rc && !dead) ? 1 : 0;
                    moved = true;
                } else {
                    const unsigned long long w =
                        __hip_atomic_load(&p.mail[e], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (w) {
                        take_mail<M::NC>(p, e, w, s.u);
                        moved = true;
                    }
                }
                if (moved) {
                    ++tcur;
                    if (tcur < tend) {
                        item = p.e2n_item[tcur];
                        trec = p.e2n_rec[tcur];
                    } else {
                        item.y = NO_STEP;
                    }
                }
                pending = item.y == b;
            }
            if (!__any(moved)) {
                if ((++spins & 255u) == 0) {
                    const bool quit = __hip_atomic_load(&p.ctrl->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ||
                                      load_error_step(p.ctrl) < (uint64_t)b;
                    // wave-uniform: every lane reads the same counter word
                    const bool late = __shfl(clock.expired(p.wait_ticks) ? 1 : 0, 0, WAVE) != 0;
                    if (late && lane == 0)
                        __hip_atomic_store(&p.ctrl->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (__any(quit) || late) break;
                    __builtin_amdgcn_s_sleep(1);
                }
            }
        }
        if constexpr (M::COUPLED) {
            const double c = coupled_sum<M>(p, s, k, b, active, owner);
            if (active && !dead) {
                if (!M::pts_coupled(s.v, s.u, s.ld, s.gd, day, c)) {
                    if (owner) raise_error(p.ctrl, b, PH_PTS, ord, E_PTS);
                    dead = true;
                }
                t.nd += owner ? 1 : 0;
            }
        } else if (active && !dead) {
            if (!M::pts(s.v, s.u, s.ld, s.gd, day)) {
                if (owner) raise_error(p.ctrl, b, PH_PTS, ord, E_PTS);
                dead = true;
            }
            t.nd += owner ? 1 : 0;
        }
        record<M>(p, s, k, run, owner, p.rec_off[b], p.rec_off[b + 1]);
    }
    add_counters(p.ctrl, t.tr, t.nd, t.ev, t.dr);
}

// ---------------------------------------------------------------------------
// barrier kernel (external transfers, several nodes per lane)
// ---------------------------------------------------------------------------
// Grid barrier on a monotone arrival counter: the epoch-th barrier completes
// when epoch * gridDim.x workgroups have arrived.
__device__ __forceinline__ void grid_barrier(Ctrl* c, unsigned epoch, uint64_t limit) {
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned target = epoch * gridDim.x;
        __hip_atomic_fetch_add(&c->bar_count, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        unsigned spins = 0;
        WaitClock clock;
        while (__hip_atomic_load(&c->bar_count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(&c->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
            if ((++spins & 255u) == 0 && clock.expired(limit)) {
                __hip_atomic_store(&c->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    __threadfence();
}

template <class M>
__device__ __forceinline__ void load_live(const KParams& p, Node<M>& s, int k) {
#pragma unroll
    for (int c = 0; c < M::NC; ++c) s.u[c] = p.u[(size_t)c * p.n + k];
#pragma unroll
    for (int c = 0; c < M::NV; ++c) s.v[c] = p.v[(size_t)c * p.n + k];
}

template <class M, bool PIPE, bool AEM = false>
__global__ void __launch_bounds__(256) sync_kernel(KParams pa) {
    KParams p = pa;
    p.seed = pa.rp->seed;
    p.stream_base = pa.rp->stream_base;
    const int lane = threadIdx.x & (WAVE - 1);
    const int gtid = blockIdx.x * blockDim.x + threadIdx.x;
    const int nthreads = gridDim.x * blockDim.x;
    const int wave_base = gtid - lane;
    Tally t;
    unsigned epoch = 0;
    for (int b = 0; b < p.nb; ++b) {
        const bool stop = error_step(p.ctrl) < (uint64_t)b;
        const int64_t day = p.T1 + b;
        const bool e2day = p.e2_step[b + 1] > p.e2_step[b];
        for (int base = wave_base; base < p.n; base += nthreads) {
            const int k = base + lane;
            const bool active = k < p.n && !stop;
            Node<M> s;
            int run = 0;
            if (active) {
                load_static<M>(p, s, k, run);
                load_live<M>(p, s, k);
                const uint32_t stream = p.stream_base + (uint32_t)run;
                const int64_t ord = p.node_ord[k];
                bool dead = false;
                int cur = p.e1_cur[k];
                const int cend = p.e1_off[k + 1];
                int4 nrec = cur < cend ? p.e1.rec[cur] : make_int4(0, 0, 0, 0);
                int wbase = cur;
                AemState<M, AEM> a{};
                if constexpr (AEM) aem_load<M>(p, k, a);
                ssa_and_e1<M, PIPE, AEM>(p, s, b, day, (uint32_t)p.node_idx[k], stream, ord, cur, cend, nrec, wbase,
                                         dead, t, false, a);
                if constexpr (AEM) aem_store<M>(p, k, a);
                p.e1_cur[k] = cur;
                if (!e2day && !dead && !M::pts(s.v, s.u, s.ld, s.gd, day))
                    raise_error(p.ctrl, b, PH_PTS, ord, E_PTS);
#pragma unroll
                for (int c = 0; c < M::NC; ++c) p.u[(size_t)c * p.n + k] = s.u[c];
                if (!e2day) {
#pragma unroll
                    for (int c = 0; c < M::NV; ++c) p.v[(size_t)c * p.n + k] = s.v[c];
                }
                ++t.nd;
            }
            if (!e2day) record<M>(p, s, k, run, active, p.rec_off[b], p.rec_off[b + 1]);
        }
        if (!e2day) continue;

        grid_barrier(p.ctrl, ++epoch, p.wait_ticks);
        if (blockIdx.x == 0) {
            // this step's transfers, level by level in key order; the branch
            // and the level loop are uniform over workgroup 0
            for (int L = p.e2_step[b]; L < p.e2_step[b + 1]; ++L) {
                for (int e = p.e2_lvl[L] + (int)threadIdx.x; e < p.e2_lvl[L + 1]; e += blockDim.x) {
                    const int src = p.e2.node[e], dst = p.e2.dest[e];
                    int32_t us[M::NC], ud[M::NC], before[M::NC];
#pragma unroll
                    for (int c = 0; c < M::NC; ++c) {
                        us[c] = p.u[(size_t)c * p.n + src];
                        ud[c] = p.u[(size_t)c * p.n + dst];
                        before[c] = ud[c];
                    }
                    const uint32_t stream = p.stream_base + (uint32_t)p.e2.run[e];
                    const int rc = apply_event<M>(p.e2.rec[e], p.e2.prop, e, p.seed, stream, us, ud);
                    if (rc) {
                        raise_error(p.ctrl, b, PH_E2, p.e2.ordinal[e], rc);
                    } else {
                        if (dst == src) {
#pragma unroll
                            for (int c = 0; c < M::NC; ++c)
                                p.u[(size_t)c * p.n + src] = us[c] + (ud[c] - before[c]);
                        } else {
#pragma unroll
                            for (int c = 0; c < M::NC; ++c) {
                                p.u[(size_t)c * p.n + src] = us[c];
                                p.u[(size_t)c * p.n + dst] = ud[c];
                            }
                        }
                        ++t.ev;
                    }
                }
                __threadfence_block();
                __syncthreads();
            }
        }
        grid_barrier(p.ctrl, ++epoch, p.wait_ticks);

        for (int base = wave_base; base < p.n; base += nthreads) {
            const int k = base + lane;
            const bool active = k < p.n && !stop;
            Node<M> s;
            int run = 0;
            if (active) {
                load_static<M>(p, s, k, run);
                load_live<M>(p, s, k);
                if (!M::pts(s.v, s.u, s.ld, s.gd, day)) raise_error(p.ctrl, b, PH_PTS, p.node_ord[k], E_PTS);
#pragma unroll
                for (int c = 0; c < M::NV; ++c) p.v[(size_t)c * p.n + k] = s.v[c];
            }
            record<M>(p, s, k, run, active, p.rec_off[b], p.rec_off[b + 1]);
        }
    }
    add_counters(p.ctrl, t.tr, t.nd, t.ev, t.dr);
}

// ---------------------------------------------------------------------------
// per-run initialisation, trajectory gather, prevalence quantiles
// ---------------------------------------------------------------------------
__global__ void init_kernel(KParams p, int nc, int nv, int first_rec, int reset_ctrl,
                            const unsigned long long* sums_init, long long sums_len) {
    const int gtid = blockIdx.x * blockDim.x + threadIdx.x;
    const int nthreads = gridDim.x * blockDim.x;
    if (reset_ctrl && gtid == 0) {
        p.ctrl->err_key = NO_ERROR;
        for (int i = 0; i < 4; ++i) p.ctrl->counters[i] = 0;
        for (int i = 0; i < MAX_GROUPS; ++i) p.ctrl->work[i] = 0;
        p.ctrl->bar_count = 0;
        p.ctrl->abort = 0;
        p.ctrl->e2done = 0;
    }
    if (reset_ctrl && sums_init)
        for (long long i = gtid; i < sums_len; i += nthreads) p.sums[i] = sums_init[i];
    if (p.mode == MODE_FLOW)
        for (int e = gtid; e < p.n_e2; e += nthreads) p.mail[e] = 0ull;
    if (p.coupled)
        for (int i = gtid; i < 2 * p.n; i += nthreads) p.cpl_post[i].day = -1;
    if (p.solver == 1) {
        // the all events method: integrals 0, each channel's first level its
        // first exponential
        const uint64_t seed = p.rp->seed;
        for (int i = gtid; i < p.nt * p.n; i += nthreads) {
            const int j = i / p.n, k = i % p.n;
            const uint32_t stream = p.rp->stream_base + (uint32_t)p.node_run[k];
            p.aem_T[i] = 0.0;
            p.aem_P[i] = aem_exp(seed, 0u, (uint32_t)j, (uint32_t)p.node_idx[k], stream);
            p.aem_K[i] = 1u;
        }
    }
    for (int k = gtid; k < p.n; k += nthreads) {
        if (p.mode == MODE_BARRIER) {
            for (int c = 0; c < nc; ++c) p.u[(size_t)c * p.n + k] = p.u0[(size_t)c * p.n + k];
            for (int c = 0; c < nv; ++c) p.v[(size_t)c * p.n + k] = p.v0[(size_t)c * p.n + k];
            p.e1_cur[k] = p.e1_off[k];
        }
        if (p.record == 0) {
            for (int m = 0; m < first_rec; ++m) {
                for (int c = 0; c < nc; ++c)
                    p.U[rec_index(m, c, k, nc, p.ntspan, p.n, p.nmajor)] = p.u0[(size_t)c * p.n + k];
                for (int c = 0; c < nv; ++c)
                    p.V[rec_index(m, c, k, nv, p.ntspan, p.n, p.nmajor)] = p.v0[(size_t)c * p.n + k];
            }
        }
    }
}

__global__ void gather_kernel(const int32_t* U, const double* V, int nc, int nv, int n, int ntspan, int nmajor,
                              const int32_t* pos, int nn, int32_t* Uo, double* Vo) {
    const long long total = (long long)ntspan * nn;
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
         idx += (long long)gridDim.x * blockDim.x) {
        const int m = (int)(idx / nn), i = (int)(idx % nn);
        const int k = pos[i];
        if (Uo)
            for (int c = 0; c < nc; ++c) Uo[((size_t)m * nn + i) * nc + c] = U[rec_index(m, c, k, nc, ntspan, n, nmajor)];
        if (Vo)
            for (int c = 0; c < nv; ++c) Vo[((size_t)m * nn + i) * nv + c] = V[rec_index(m, c, k, nv, ntspan, n, nmajor)];
    }
}

// Sparse copy-out (Table 1, U_sparse / V_sparse): entry e of a compressed-
// column pattern over the (Nn*width) x Ntspan matrix (column m = tspan
// index, row = node*width + c) takes the recorded value, as binary64.
__global__ void sparse_gather_kernel(const int32_t* U, const double* V, int width, int n, int ntspan, int nmajor,
                                     const int32_t* pos, const int64_t* col_ptr, const int32_t* row_idx,
                                     long long nnz, double* out) {
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nnz;
         e += (long long)gridDim.x * blockDim.x) {
        // the column of entry e: the last m with col_ptr[m] <= e
        int lo = 0, hi = ntspan;
        while (hi - lo > 1) {
            const int mid = (lo + hi) / 2;
            if (col_ptr[mid] <= e)
                lo = mid;
            else
                hi = mid;
        }
        const int row = row_idx[e];
        const int k = pos[row / width], c = row % width;
        const size_t at = rec_index(lo, c, k, width, ntspan, n, nmajor);
        out[e] = U ? (double)U[at] : V[at];
    }
}

// One workgroup per (set, tspan index): prevalence of every replicate, rank
// sort (ties by replicate index), type-7 quantiles.
__global__ void prevalence_kernel(const unsigned long long* sums, int ntspan, int nc, int case_c, uint32_t mask,
                                  int reps, int k0, int nk, const double* probs, int nq, float* out) {
    extern __shared__ double sh[];
    double* val = sh;
    double* sorted = sh + reps;
    const int set = blockIdx.x / nk, kk = blockIdx.x % nk;
    const int k = k0 + kk;
    for (int r = threadIdx.x; r < reps; r += blockDim.x) {
        const int run = set * reps + r;
        const long long* row = (const long long*)sums + ((size_t)run * ntspan + k) * nc;
        long long den = 0;
        for (int c = 0; c < nc; ++c)
            if ((mask >> c) & 1u) den += row[c];
        val[r] = den > 0 ? (double)row[case_c] / (double)den : 0.0;
    }
    __syncthreads();
    for (int r = threadIdx.x; r < reps; r += blockDim.x) {
        const double x = val[r];
        int rank = 0;
        for (int o = 0; o < reps; ++o) rank += (val[o] < x) || (val[o] == x && o < r);
        sorted[rank] = x;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < nq; q += blockDim.x) {
        const double h = (double)(reps - 1) * probs[q];
        const double fl = floor(h);
        const int lo = (int)fl;
        const double frac = h - fl;
        double res = sorted[lo];
        if (lo + 1 < reps) res = sorted[lo] + (sorted[lo + 1] - sorted[lo]) * frac;
        out[((size_t)set * nk + kk) * nq + q] = (float)res;
    }
}

#ifndef __HIPCC_RTC__
template <class M, bool PIPE>
const void* kernel_for(int mode, bool grp) {
    // nodes on groups of lanes have their own instantiations, so that the
    // other launches keep the register budget they need
    if (mode == MODE_FLOW) return grp ? (const void*)flow_kernel<M, PIPE, true> : (const void*)flow_kernel<M, PIPE, false>;
    if (mode == MODE_BARRIER) return (const void*)sync_kernel<M, PIPE>;
    return grp ? (const void*)free_kernel<M, PIPE, true> : (const void*)free_kernel<M, PIPE, false>;
}

template <class M>
const void* kernel_for(int mode, int pipeline, bool grp, bool lq, bool aem) {
    if (aem) {
        // the all events method: one lane per node
        if (grp || lq) return nullptr;
        if (mode == MODE_FLOW) return (const void*)flow_kernel<M, false, false, true>;
        if (mode == MODE_BARRIER) return (const void*)sync_kernel<M, false, true>;
        return (const void*)free_kernel<M, false, false, true>;
    }
    if (mode == MODE_FREE && lq) return pipeline ? (const void*)lane_kernel<M, true> : (const void*)lane_kernel<M, false>;
    return pipeline ? kernel_for<M, true>(mode, grp) : kernel_for<M, false>(mode, grp);
}

const void* model_kernel(int model, int mode, int pipeline, bool grp, bool lq, bool aem) {
    switch (model) {
        case M_SIR: return kernel_for<ModelSIR>(mode, pipeline, grp, lq, aem);
        case M_SIS: return kernel_for<ModelSIS>(mode, pipeline, grp, lq, aem);
        case M_SISE: return kernel_for<ModelSISe>(mode, pipeline, grp, lq, aem);
        case M_BIRTH_DEATH: return kernel_for<ModelBirthDeath>(mode, pipeline, grp, lq, aem);
        case M_IMMIGRATION_DEATH: return kernel_for<ModelImmigrationDeath>(mode, pipeline, grp, lq, aem);
        case M_SISE_SP:
            // the coupled post-time step exists in the dataflow kernel only
            if (mode != MODE_FLOW || lq) return nullptr;
            if (aem) return grp ? nullptr : (const void*)flow_kernel<ModelSISeSp, false, false, true>;
            if (pipeline)
                return grp ? (const void*)flow_kernel<ModelSISeSp, true, true>
                           : (const void*)flow_kernel<ModelSISeSp, true, false>;
            return grp ? (const void*)flow_kernel<ModelSISeSp, false, true>
                       : (const void*)flow_kernel<ModelSISeSp, false, false>;
    }
    return nullptr;
}

#endif  // __HIPCC_RTC__

}  // namespace

#ifndef __HIPCC_RTC__
hipError_t launch_init(const KParams& p, int nc, int nv, int first_rec, bool reset_ctrl,
                       const unsigned long long* sums_init, long long sums_len, hipStream_t st) {
    int blocks = (int)((std::max(p.coupled ? 2 * p.n : p.n, p.n_e2) + 255) / 256);
    if (sums_init) blocks = (int)std::max<long long>(blocks, (sums_len + 255) / 256);
    blocks = std::max(1, std::min(blocks, 4096));
    init_kernel<<<blocks, 256, 0, st>>>(p, nc, nv, first_rec, reset_ctrl ? 1 : 0, sums_init, sums_len);
    return hipGetLastError();
}

hipError_t launch_group(int model, const KParams& p, int block, int blocks, size_t shmem, hipStream_t st) {
    if (model >= SIMINF_GEN_FIRST) return generated_launch(model, p, block, blocks, shmem, st);
    const void* fn = model_kernel(model, p.mode, p.pipeline, p.ngrp > 0, p.lane_queue != 0, p.solver == 1);
    if (!fn) return hipErrorInvalidValue;
    KParams arg = p;
    void* args[] = {&arg};
    if (p.mode == MODE_FREE) return hipLaunchKernel(fn, dim3(blocks), dim3(block), args, shmem, st);
    return hipLaunchCooperativeKernel(fn, dim3(blocks), dim3(block), args, (unsigned)shmem, st);
}

int max_blocks_per_cu(int model, int mode, int pipeline, bool grp, int block, size_t shmem, bool lane_queue,
                      bool aem) {
    if (model >= SIMINF_GEN_FIRST)
        return grp || lane_queue ? 0 : generated_blocks_per_cu(model, mode, pipeline, block, shmem, aem);
    const void* fn = model_kernel(model, mode, pipeline, grp, lane_queue, aem);
    int n = 0;
    if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, block, shmem) != hipSuccess) return 0;
    return n;
}

hipError_t launch_gather(int nc, int nv, const int32_t* U, const double* V, int n, int ntspan, int nmajor,
                         const int32_t* pos, int nn, int32_t* Uo, double* Vo, hipStream_t st) {
    long long total = (long long)ntspan * nn;
    int blocks = (int)std::max<long long>(1, std::min<long long>((total + 255) / 256, 8192));
    gather_kernel<<<blocks, 256, 0, st>>>(U, V, nc, nv, n, ntspan, nmajor, pos, nn, Uo, Vo);
    return hipGetLastError();
}

hipError_t launch_sparse_gather(const int32_t* U, const double* V, int width, int n, int ntspan, int nmajor,
                                const int32_t* pos, const int64_t* col_ptr, const int32_t* row_idx, long long nnz,
                                double* out, hipStream_t st) {
    if (nnz <= 0) return hipSuccess;
    const int blocks = (int)std::max<long long>(1, std::min<long long>((nnz + 255) / 256, 8192));
    sparse_gather_kernel<<<blocks, 256, 0, st>>>(U, V, width, n, ntspan, nmajor, pos, col_ptr, row_idx, nnz, out);
    return hipGetLastError();
}

hipError_t launch_prevalence(const unsigned long long* sums, int runs, int ntspan, int nc, int case_c, uint32_t mask,
                             int reps, int k0, int nk, const double* probs, int nq, float* out, hipStream_t st) {
    const int sets = runs / reps;
    if (sets <= 0 || nk <= 0) return hipSuccess;
    const size_t shmem = sizeof(double) * 2 * (size_t)reps;
    prevalence_kernel<<<sets * nk, 64, shmem, st>>>(sums, ntspan, nc, case_c, mask, reps, k0, nk, probs, nq, out);
    return hipGetLastError();
}

#endif  // __HIPCC_RTC__

}  // namespace siminf
