// ssa_kernels.hip -- gfx950 kernels of the split-step direct-method SSA
// (section 2.3 and Appendix A of arXiv 1605.01421): one lane per node.
//
// Two persistent kernels per model:
//  * free_kernel: used when the run has no external transfers.  Nodes are
//    then independent for the whole run, so each wavefront takes 64-node
//    chunks from a work queue and carries every node through all days with
//    the state in registers; no grid-wide synchronisation at all.
//  * sync_kernel: used when external transfers exist.  Launched
//    cooperatively (all workgroups resident); every day all lanes run SSA +
//    E1 for their nodes, and on days with external transfers a grid barrier
//    is followed by workgroup 0 applying that day's transfers level by level
//    (events of one level touch disjoint nodes), a second barrier, and the
//    post-time step.
#include "device_math.h"
#include "internal.h"
#include "models.h"

#include <algorithm>

namespace siminf {

namespace {

constexpr int E_NEG_STATE = -5, E_BAD_RATE = -6, E_OVERDRAW = -7, E_PTS = -9, E_DEVICE = -4;
constexpr int EV_EXIT = 0, EV_ENTER = 1, EV_EXTTRANS = 3;
constexpr unsigned SPIN_LIMIT = 1u << 22;
// Transitions of one node within one unit of time beyond which the rates are
// declared unusable (time would no longer advance at binary64 resolution).
constexpr uint32_t STEP_LIMIT = 1u << 24;

__device__ __forceinline__ void raise_error(Ctrl* c, int step, int phase, int64_t ord, int code) {
    atomicMin(&c->err_key, make_err_key((uint32_t)step, (uint32_t)phase, (uint64_t)ord, (uint32_t)(-code)));
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, WAVE);
    return x;
}

// First step index whose error stops further work (wave-uniform).
__device__ __forceinline__ uint64_t error_step(Ctrl* c) {
    uint64_t k = 0;
    if ((threadIdx.x & (WAVE - 1)) == 0)
        k = __hip_atomic_load(&c->err_key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    k = __shfl(k, 0, WAVE);
    return k >> 44;
}

template <class M>
struct Node {
    int32_t u[M::NC];
    double v[M::NV > 0 ? M::NV : 1];
    double ld[M::NLD > 0 ? M::NLD : 1];
    double gd[M::NGD];
};

template <class M>
__device__ __forceinline__ bool rate_ok(double w) {
    return w >= 0.0 && isfinite(w);
}

// Direct-method SSA of one node from time t to the day boundary T
// (Appendix A, lines 8-19).  Returns 0 or an error code.
template <class M>
__device__ __forceinline__ int ssa_to_boundary(const KParams& p, Node<M>& s, double t, double T,
                                               uint32_t day_word, uint32_t node, uint32_t stream,
                                               unsigned long long& transitions,
                                               unsigned long long& draws) {
    static_assert(M::NT == 2, "kernels are written for two-transition models");
    double w0 = M::template rate<0>(s.u, s.v, s.ld, s.gd);
    double w1 = M::template rate<1>(s.u, s.v, s.ld, s.gd);
    if (!rate_ok<M>(w0) || !rate_ok<M>(w1)) return E_BAD_RATE;
    const uint32_t k0 = (uint32_t)p.seed, k1 = (uint32_t)(p.seed >> 32);
    const uint32_t tag = stream & 0xFFFFFFu;
    for (uint32_t step = 0;; ++step) {
        double lam = 0.0;
        lam = lam + w0;
        lam = lam + w1;
        if (!(lam > 0.0)) break;
        if (step == STEP_LIMIT) return E_BAD_RATE;
        draws += 1;
        const Block4 r = philox10(k0, k1, step, day_word, node, tag);
        const double r1 = open_uniform(r.x, r.y);
        const double r2 = open_uniform(r.z, r.w);
        const double tau = (-series_log(r1)) / lam;
        const double tn = t + tau;
        if (tn >= T) break;
        t = tn;
        // inversion: first transition with positive rate whose cumulative
        // sum reaches lam*r2; the running sum after the first rate is w0.
        const double x = lam * r2;
        const int n = (w0 > 0.0 && x <= w0) ? 0 : (w1 > 0.0 ? 1 : 0);
        bool neg = false;
#pragma unroll
        for (int c = 0; c < M::NC; ++c) {
            s.u[c] += n ? p.S[c + M::NC] : p.S[c];
            neg |= s.u[c] < 0;
        }
        transitions += 1;
        if (neg) return E_NEG_STATE;
        const uint32_t g = n ? p.Gmask[1] : p.Gmask[0];
        if (g & 1u) w0 = M::template rate<0>(s.u, s.v, s.ld, s.gd);
        if (g & 2u) w1 = M::template rate<1>(s.u, s.v, s.ld, s.gd);
        if (!rate_ok<M>(w0) || !rate_ok<M>(w1)) return E_BAD_RATE;
    }
    return 0;
}

// One scheduled event (section 3.3) on node state u (and destination ud for
// an external transfer).  Indices were validated when the model was created.
// Returns 0 or E_OVERDRAW; on error the states are unchanged.
template <int NC>
__device__ __forceinline__ int apply_event(const KParams& p, const EventSoA& ev, int e, int32_t (&u)[NC],
                                        int32_t (&ud)[NC], uint32_t stream) {
    const int type = ev.type[e];
    const uint32_t mask = p.Emask[ev.select[e]];
    if (type == EV_ENTER) {
        // all n individuals go to the first selected compartment
        bool done = false;
#pragma unroll
        for (int c = 0; c < NC; ++c)
            if (!done && ((mask >> c) & 1u)) {
                u[c] += ev.n[e];
                done = true;
            }
        return 0;
    }
    const int q = ev.shift[e];
    int tgt[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) tgt[c] = q >= 0 ? c + p.Nshift[q * MAX_NC + c] : c;
    int64_t total = 0;
#pragma unroll
    for (int c = 0; c < NC; ++c)
        if ((mask >> c) & 1u) total += u[c];
    int64_t n = ev.n[e];
    if (n == 0) n = (int64_t)floor(ev.prop[e] * (double)total + 0.5);
    if (n > total) return E_OVERDRAW;
    int32_t take[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) take[c] = (n == total && ((mask >> c) & 1u)) ? u[c] : 0;
    if (n < total) {
        EventWords words(p.seed, stream, (uint32_t)ev.id[e]);
        for (int64_t k = 0; k < n; ++k) {
            const int64_t j = words.below((uint32_t)(total - k));
            int64_t below = 0;
            bool hit = false;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                if ((mask >> c) & 1u) {
                    below += u[c] - take[c];
                    if (!hit && j < below) {
                        take[c] += 1;
                        hit = true;
                    }
                }
            }
        }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) u[c] -= take[c];
    if (type == EV_EXIT) return 0;
    const bool ext = type == EV_EXTTRANS;
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int d = 0; d < NC; ++d)
            if (tgt[c] == d) {
                if (ext)
                    ud[d] += take[c];
                else
                    u[d] += take[c];
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

// Writes the records of tspan indices [m0, m1) (all lanes of the wave call
// this together; inactive lanes contribute nothing).
template <class M>
__device__ __forceinline__ void record(const KParams& p, const Node<M>& s, int k, int run, bool active,
                                       int m0, int m1) {
    for (int m = m0; m < m1; ++m) {
        if (p.record == 0) {
            if (active) {
#pragma unroll
                for (int c = 0; c < M::NC; ++c) p.U[((size_t)m * M::NC + c) * p.n + k] = s.u[c];
#pragma unroll
                for (int c = 0; c < M::NV; ++c) p.V[((size_t)m * M::NV + c) * p.n + k] = s.v[c];
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
                unsigned long long* dst = p.sums + ((size_t)run * p.ntspan + m) * p.sums_nc + c;
                if (same) {
                    const unsigned long long tot = wave_sum(val);
                    if (lane == leader)
                        atomicAdd(p.sums + ((size_t)run0 * p.ntspan + m) * p.sums_nc + c, tot);
                } else if (active) {
                    atomicAdd(dst, val);
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

// ---------------------------------------------------------------------------
// free-running kernel (no external transfers)
// ---------------------------------------------------------------------------
template <class M>
__global__ void __launch_bounds__(256) free_kernel(KParams p) {
    const int lane = threadIdx.x & (WAVE - 1);
    unsigned long long n_tr = 0, n_nd = 0, n_ev = 0, n_dr = 0;
    for (;;) {
        unsigned chunk = 0;
        if (lane == 0) chunk = atomicAdd(&p.ctrl->work[p.group], 1u);
        chunk = __shfl(chunk, 0, WAVE);
        if (chunk >= (unsigned)p.nchunks) break;
        const int k = (int)chunk * WAVE + lane;
        const bool active = k < p.n;
        Node<M> s;
        int run = 0, cur = 0, cend = 0;
        uint32_t node = 0, stream = 0;
        int64_t ord = 0;
        if (active) {
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
        }
        bool dead = false;
        for (int b = 0; b < p.nb; ++b) {
            if (error_step(p.ctrl) < (uint64_t)b) break;
            const int64_t day = p.T1 + b;
            const double T = (double)day;
            const double t = b == 0 ? p.t0 : T - 1.0;
            if (active && !dead) {
                int rc = ssa_to_boundary<M>(p, s, t, T, (uint32_t)(int32_t)day, node, stream, n_tr, n_dr);
                if (rc) {
                    raise_error(p.ctrl, b, PH_SSA, ord, rc);
                    dead = true;
                }
                while (!dead && cur < cend && (double)p.e1.time[cur] <= T) {
                    rc = apply_event<M::NC>(p, p.e1, cur, s.u, s.u, stream);
                    if (rc) {
                        raise_error(p.ctrl, b, PH_E1, p.e1.ordinal[cur], rc);
                        dead = true;
                    } else {
                        ++n_ev;
                        ++cur;
                    }
                }
                if (!dead && !M::pts(s.v, s.u, s.ld, s.gd, day)) {
                    raise_error(p.ctrl, b, PH_PTS, ord, E_PTS);
                    dead = true;
                }
                ++n_nd;
            }
            record<M>(p, s, k, run, active, p.rec_off[b], p.rec_off[b + 1]);
        }
    }
    add_counters(p.ctrl, n_tr, n_nd, n_ev, n_dr);
}

// ---------------------------------------------------------------------------
// day-synchronous kernel (external transfers present); cooperative launch
// ---------------------------------------------------------------------------
// Grid barrier on a monotone arrival counter: the epoch-th barrier completes
// when epoch * gridDim.x workgroups have arrived.  A wait that exceeds the
// spin limit sets `abort`, after which every barrier returns at once (the run
// then reports SIMINF_E_DEVICE) so the kernel always terminates.
__device__ __forceinline__ void grid_barrier(Ctrl* c, unsigned epoch) {
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned target = epoch * gridDim.x;
        __hip_atomic_fetch_add(&c->bar_count, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        unsigned spins = 0;
        while (__hip_atomic_load(&c->bar_count, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(&c->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
            if (++spins > SPIN_LIMIT) {
                __hip_atomic_store(&c->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            __builtin_amdgcn_s_sleep(4);
        }
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

template <class M>
__global__ void __launch_bounds__(256) sync_kernel(KParams p) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int gtid = blockIdx.x * blockDim.x + threadIdx.x;
    const int nthreads = gridDim.x * blockDim.x;
    const int wave_base = gtid - lane;
    unsigned long long n_tr = 0, n_nd = 0, n_ev = 0, n_dr = 0;
    unsigned epoch = 0;
    for (int b = 0; b < p.nb; ++b) {
        const bool stop = error_step(p.ctrl) < (uint64_t)b;
        const int64_t day = p.T1 + b;
        const double T = (double)day;
        const double t = b == 0 ? p.t0 : T - 1.0;
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
                int rc = ssa_to_boundary<M>(p, s, t, T, (uint32_t)(int32_t)day, (uint32_t)p.node_idx[k],
                                            stream, n_tr, n_dr);
                if (rc) {
                    raise_error(p.ctrl, b, PH_SSA, ord, rc);
                    dead = true;
                }
                int cur = p.e1_cur[k];
                const int cend = p.e1_off[k + 1];
                while (!dead && cur < cend && (double)p.e1.time[cur] <= T) {
                    rc = apply_event<M::NC>(p, p.e1, cur, s.u, s.u, stream);
                    if (rc) {
                        raise_error(p.ctrl, b, PH_E1, p.e1.ordinal[cur], rc);
                        dead = true;
                    } else {
                        ++n_ev;
                        ++cur;
                    }
                }
                p.e1_cur[k] = cur;
                if (!e2day && !dead && !M::pts(s.v, s.u, s.ld, s.gd, day))
                    raise_error(p.ctrl, b, PH_PTS, ord, E_PTS);
#pragma unroll
                for (int c = 0; c < M::NC; ++c) p.u[(size_t)c * p.n + k] = s.u[c];
                if (!e2day) {
#pragma unroll
                    for (int c = 0; c < M::NV; ++c) p.v[(size_t)c * p.n + k] = s.v[c];
                }
                ++n_nd;
            }
            if (!e2day) record<M>(p, s, k, run, active, p.rec_off[b], p.rec_off[b + 1]);
        }
        if (!e2day) continue;

        grid_barrier(p.ctrl, ++epoch);
        if (blockIdx.x == 0) {
            // external transfers of this step, level by level, in key order;
            // the branch and the level loop are uniform over workgroup 0
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
                    const uint32_t stream = p.stream_base + (uint32_t)p.node_run[src];
                    const int rc = apply_event<M::NC>(p, p.e2, e, us, ud, stream);
                    if (rc) {
                        raise_error(p.ctrl, b, PH_E2, p.e2.ordinal[e], rc);
                    } else {
                        if (dst == src) {
                            // one node: removal and (shifted) re-addition both apply
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
                        ++n_ev;
                    }
                }
                __threadfence_block();
                __syncthreads();
            }
        }
        grid_barrier(p.ctrl, ++epoch);

        for (int base = wave_base; base < p.n; base += nthreads) {
            const int k = base + lane;
            const bool active = k < p.n && !stop;
            Node<M> s;
            int run = 0;
            if (active) {
                load_static<M>(p, s, k, run);
                load_live<M>(p, s, k);
                if (!M::pts(s.v, s.u, s.ld, s.gd, day))
                    raise_error(p.ctrl, b, PH_PTS, p.node_ord[k], E_PTS);
#pragma unroll
                for (int c = 0; c < M::NV; ++c) p.v[(size_t)c * p.n + k] = s.v[c];
            }
            record<M>(p, s, k, run, active, p.rec_off[b], p.rec_off[b + 1]);
        }
    }
    add_counters(p.ctrl, n_tr, n_nd, n_ev, n_dr);
    if (gtid == 0 && __hip_atomic_load(&p.ctrl->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        raise_error(p.ctrl, 0, 0, 0, E_DEVICE);
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
    }
    if (reset_ctrl && sums_init)
        for (long long i = gtid; i < sums_len; i += nthreads) p.sums[i] = sums_init[i];
    for (int k = gtid; k < p.n; k += nthreads) {
        if (p.mode == 1) {
            for (int c = 0; c < nc; ++c) p.u[(size_t)c * p.n + k] = p.u0[(size_t)c * p.n + k];
            for (int c = 0; c < nv; ++c) p.v[(size_t)c * p.n + k] = p.v0[(size_t)c * p.n + k];
            p.e1_cur[k] = p.e1_off[k];
        }
        if (p.record == 0) {
            for (int m = 0; m < first_rec; ++m) {
                for (int c = 0; c < nc; ++c)
                    p.U[((size_t)m * nc + c) * p.n + k] = p.u0[(size_t)c * p.n + k];
                for (int c = 0; c < nv; ++c)
                    p.V[((size_t)m * nv + c) * p.n + k] = p.v0[(size_t)c * p.n + k];
            }
        }
    }
}

__global__ void gather_kernel(const int32_t* U, const double* V, int nc, int nv, int n, int ntspan,
                              const int32_t* pos, int nn, int32_t* Uo, double* Vo) {
    const long long total = (long long)ntspan * nn;
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
         idx += (long long)gridDim.x * blockDim.x) {
        const int m = (int)(idx / nn), i = (int)(idx % nn);
        const int k = pos[i];
        if (Uo)
            for (int c = 0; c < nc; ++c)
                Uo[((size_t)m * nn + i) * nc + c] = U[((size_t)m * nc + c) * n + k];
        if (Vo)
            for (int c = 0; c < nv; ++c)
                Vo[((size_t)m * nn + i) * nv + c] = V[((size_t)m * nv + c) * n + k];
    }
}

// One workgroup per (set, tspan index): prevalence of every replicate, rank
// sort (ties by replicate index), type-7 quantiles.
__global__ void prevalence_kernel(const unsigned long long* sums, int ntspan, int nc, int case_c,
                                  uint32_t mask, int reps, int k0, int nk, const double* probs, int nq,
                                  float* out) {
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

template <class M>
hipError_t launch_model(const KParams& p, int block, int blocks, bool cooperative, hipStream_t st) {
    if (cooperative) {
        KParams arg = p;
        void* args[] = {&arg};
        return hipLaunchCooperativeKernel((const void*)sync_kernel<M>, dim3(blocks), dim3(block), args, 0, st);
    }
    free_kernel<M><<<blocks, block, 0, st>>>(p);
    return hipGetLastError();
}

template <class M>
int occupancy(int mode, int block) {
    int n = 0;
    hipError_t e = mode == 1
        ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, sync_kernel<M>, block, 0)
        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, free_kernel<M>, block, 0);
    return e == hipSuccess ? n : 0;
}

}  // namespace

hipError_t launch_init(const KParams& p, int nc, int nv, int first_rec, bool reset_ctrl,
                       const unsigned long long* sums_init, long long sums_len, hipStream_t st) {
    int blocks = (int)((p.n + 255) / 256);
    if (sums_init) blocks = (int)std::max<long long>(blocks, (sums_len + 255) / 256);
    blocks = std::max(1, std::min(blocks, 4096));
    init_kernel<<<blocks, 256, 0, st>>>(p, nc, nv, first_rec, reset_ctrl ? 1 : 0, sums_init, sums_len);
    return hipGetLastError();
}

hipError_t launch_group(int model, const KParams& p, int block, int blocks, bool cooperative,
                        hipStream_t st) {
    switch (model) {
        case M_SIR: return launch_model<ModelSIR>(p, block, blocks, cooperative, st);
        case M_SIS: return launch_model<ModelSIS>(p, block, blocks, cooperative, st);
        case M_SISE: return launch_model<ModelSISe>(p, block, blocks, cooperative, st);
        case M_BIRTH_DEATH: return launch_model<ModelBirthDeath>(p, block, blocks, cooperative, st);
        case M_IMMIGRATION_DEATH:
            return launch_model<ModelImmigrationDeath>(p, block, blocks, cooperative, st);
    }
    return hipErrorInvalidValue;
}

int max_blocks_per_cu(int model, int mode, int block) {
    switch (model) {
        case M_SIR: return occupancy<ModelSIR>(mode, block);
        case M_SIS: return occupancy<ModelSIS>(mode, block);
        case M_SISE: return occupancy<ModelSISe>(mode, block);
        case M_BIRTH_DEATH: return occupancy<ModelBirthDeath>(mode, block);
        case M_IMMIGRATION_DEATH: return occupancy<ModelImmigrationDeath>(mode, block);
    }
    return 0;
}

hipError_t launch_gather(int nc, int nv, const int32_t* U, const double* V, int n, int ntspan,
                         const int32_t* pos, int nn, int32_t* Uo, double* Vo, hipStream_t st) {
    long long total = (long long)ntspan * nn;
    int blocks = (int)std::max<long long>(1, std::min<long long>((total + 255) / 256, 8192));
    gather_kernel<<<blocks, 256, 0, st>>>(U, V, nc, nv, n, ntspan, pos, nn, Uo, Vo);
    return hipGetLastError();
}

hipError_t launch_prevalence(const unsigned long long* sums, int runs, int ntspan, int nc, int case_c,
                             uint32_t mask, int reps, int k0, int nk, const double* probs, int nq,
                             float* out, hipStream_t st) {
    const int sets = runs / reps;
    if (sets <= 0 || nk <= 0) return hipSuccess;
    const size_t shmem = sizeof(double) * 2 * (size_t)reps;
    prevalence_kernel<<<sets * nk, 64, shmem, st>>>(sums, ntspan, nc, case_c, mask, reps, k0, nk, probs,
                                                    nq, out);
    return hipGetLastError();
}

}  // namespace siminf
