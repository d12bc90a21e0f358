// runtime.cpp -- host side of libsiminf.so: validation, layout of a run (or a
// batch of runs) in device memory, event tables, launch configuration and the
// C ABI declared in include/siminf.h.
#include "siminf.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <string>
#include <tuple>
#include <vector>

#include "internal.h"
#include "models.h"

using namespace siminf;

namespace siminf {
// generated models (generated.cpp)
bool generated_shape(int id, ModelShape* s);
int generated_check_spec(const siminf_spec& s);
}  // namespace siminf

namespace {

bool is_generated(int model) { return model >= SIMINF_GEN_FIRST && model <= SIMINF_GEN_LAST; }

bool shape_of(int model, ModelShape* s) { return model_shape(model, s) || (is_generated(model) && generated_shape(model, s)); }

struct RunInfo {
    int spec;
    int group;
    int64_t noff;  // global ordinal of the run's node 0
    int32_t nn;
    int64_t eoff;  // global ordinal of the run's event 0
};

struct Group {
    int model = 0;
    ModelShape shape{};
    int n = 0;
    int mode = 0;  // 0 free-running, 1 day-synchronous
    int block = 256, blocks = 1;
    size_t shmem = 0;
    KParams p{};
    int64_t n_e1 = 0, n_e2 = 0, n_levels = 0;
    std::vector<int64_t> work;  // expected work of each node, internal (descending) order
    std::vector<int32_t> node_run;  // run of each node, internal order (lane-queue chunks)
    int4* d_chunks = nullptr;       // lane-queue chunk table and its capacity
    int chunk_cap = 0;
    int lq_chunk = 0;               // lane queue: nodes per chunk (0 = off)
    int lq_batch = 0;               //             lanes per day-end batch
};

template <class T>
hipError_t to_device(std::vector<void*>& owned, const std::vector<T>& h, T** d) {
    *d = nullptr;
    size_t bytes = sizeof(T) * std::max<size_t>(h.size(), 1);
    hipError_t e = hipMalloc((void**)d, bytes);
    if (e != hipSuccess) return e;
    owned.push_back((void*)*d);
    if (!h.empty()) e = hipMemcpy(*d, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice);
    return e;
}

template <class T>
hipError_t alloc_device(std::vector<void*>& owned, size_t count, T** d) {
    *d = nullptr;
    hipError_t e = hipMalloc((void**)d, sizeof(T) * std::max<size_t>(count, 1));
    if (e == hipSuccess) owned.push_back((void*)*d);
    return e;
}

}  // namespace

struct siminf_model {
    int device = 0;
    std::vector<void*> owned;
    int nspec = 0, R = 0;
    std::vector<RunInfo> runs;
    int ntspan = 0, nb = 0, first_rec = 0;
    double t0 = 0;
    int64_t T1 = 0;
    std::vector<int32_t> rec_off;
    int record = 0, ncmax = 0, nvmax = 0;
    int64_t total_nodes = 0, total_events = 0;
    std::vector<Group> groups;
    Ctrl* d_ctrl = nullptr;
    unsigned long long *d_sums = nullptr, *d_sums_init = nullptr;
    long long sums_len = 0;
    int32_t* d_pos = nullptr;
    hipStream_t last_stream = nullptr;
    void* stage = nullptr;  // siminf_trajectory's device staging for host copies
    size_t stage_bytes = 0;
    bool pending = false, ran = false;
    int status = 0;
    int32_t err_code = 0, err_phase = -1, err_run = -1;
    int64_t err_step = -1, err_index = -1;
    uint64_t counters[4] = {0, 0, 0, 0};
    siminf_options opt{};
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};  // run start, SSA kernels start, run end
    RunParams* d_rp = nullptr;  // the run's seed and stream base, read by the kernels
    RunParams* h_rp = nullptr;  // pinned host staging of d_rp
    hipGraph_t graph = nullptr;  // options.graph: the captured init and SSA launches
    hipGraphExec_t gexec = nullptr;
    // model groups after the first run on side streams, forked from and
    // joined back into the run's stream, so that their kernels overlap
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> joins;
    hipEvent_t fork = nullptr;
};

namespace {

// Drops the captured launch sequence (the launch configuration changed).
void drop_graph(siminf_model* m) {
    if (m->gexec) (void)hipGraphExecDestroy(m->gexec);
    if (m->graph) (void)hipGraphDestroy(m->graph);
    m->gexec = nullptr;
    m->graph = nullptr;
}

int hip_fail(siminf_model* m) {
    if (m) m->status = SIMINF_E_DEVICE;
    return SIMINF_E_DEVICE;
}

void set_create_error(siminf_model* m, int code, int64_t index, int run) {
    m->err_code = code;
    m->err_step = -1;
    m->err_phase = -1;
    m->err_index = index;
    m->err_run = run;
    m->status = code;
}

// Static validity check of one spec (section 3.4.2).  Returns 0 or a code;
// *bad_event receives the offending event's input index (or -1).
int validate_spec(const siminf_spec& s, int64_t* bad_event) {
    *bad_event = -1;
    ModelShape sh;
    if (!shape_of(s.model, &sh)) return SIMINF_E_UNSUPPORTED;
    if (s.Nc != sh.nc || s.Nt != sh.nt) return SIMINF_E_ARG;
    if (s.Nv != sh.nv || s.Nld < sh.nld || s.Ngd < sh.ngd) return SIMINF_E_ARG;
    if (s.Nn < 0 || s.Ntspan < 1 || s.Nev < 0 || s.Ecols < 0 || s.Ncols < 0) return SIMINF_E_ARG;
    if (!s.S || !s.G || !s.tspan || (s.Nn > 0 && !s.u0)) return SIMINF_E_ARG;
    if (sh.ngd > 0 && !s.gdata) return SIMINF_E_ARG;
    if (s.Nn > 0 && s.Nv > 0 && !s.v0) return SIMINF_E_ARG;
    if (s.Nn > 0 && s.Nld > 0 && !s.ldata) return SIMINF_E_ARG;
    for (int k = 0; k < s.Ntspan; ++k)
        if (!std::isfinite(s.tspan[k]) || (k > 0 && !(s.tspan[k] > s.tspan[k - 1]))) return SIMINF_E_ARG;
    if (s.model == M_SISE_SP) {
        // the sparse distance matrix: compressed columns within the run
        if (!s.nb_ptr || s.Nnb < 0 || (s.Nnb > 0 && (!s.nb_idx || !s.nb_dist)) || s.nb_ptr[0] != 0 ||
            s.nb_ptr[s.Nn] != s.Nnb)
            return SIMINF_E_ARG;
        for (int i = 0; i < s.Nn; ++i)
            if (s.nb_ptr[i + 1] < s.nb_ptr[i]) return SIMINF_E_ARG;
        for (int e = 0; e < s.Nnb; ++e)
            if (s.nb_idx[e] < 0 || s.nb_idx[e] >= s.Nn || !(s.nb_dist[e] > 0.0) || !std::isfinite(s.nb_dist[e]))
                return SIMINF_E_ARG;
    }
    for (int64_t i = 0; i < (int64_t)s.Nn * s.Nc; ++i)
        if (s.u0[i] < 0) return SIMINF_E_ARG;
    if (s.Nev > 0) {
        if (!s.ev_type || !s.ev_time || !s.ev_node || !s.ev_dest || !s.ev_n || !s.ev_select ||
            !s.ev_shift || !s.ev_prop)
            return SIMINF_E_ARG;
        if (s.Ecols > 0 && !s.E) return SIMINF_E_ARG;
        if (s.Ncols > 0 && !s.N) return SIMINF_E_ARG;
    }
    if (is_generated(s.model)) {
        // S, G and the event tables are the model's own
        const int rc = generated_check_spec(s);
        if (rc) return rc;
    }
    for (int e = 0; e < s.Nev; ++e) {
        const int ty = s.ev_type[e];
        bool ok = ty >= SIMINF_EXIT && ty <= SIMINF_EXTTRANS;
        ok = ok && s.ev_node[e] >= 0 && s.ev_node[e] < s.Nn;
        ok = ok && (ty != SIMINF_EXTTRANS || (s.ev_dest[e] >= 0 && s.ev_dest[e] < s.Nn));
        ok = ok && s.ev_select[e] >= 0 && s.ev_select[e] < s.Ecols;
        ok = ok && s.ev_n[e] >= 0;
        ok = ok && s.ev_shift[e] >= -1 && s.ev_shift[e] < s.Ncols;
        ok = ok && std::isfinite(s.ev_prop[e]) && s.ev_prop[e] >= 0.0 && s.ev_prop[e] <= 1.0;
        if (ok) {
            const int32_t* Ecol = s.E + (size_t)s.ev_select[e] * s.Nc;
            bool any = false;
            for (int c = 0; c < s.Nc; ++c) {
                if (!Ecol[c]) continue;
                any = true;
                if (ty != SIMINF_ENTER && s.ev_shift[e] >= 0) {
                    const int t = c + s.N[(size_t)s.ev_shift[e] * s.Nc + c];
                    if (t < 0 || t >= s.Nc) ok = false;
                }
            }
            if (ty == SIMINF_ENTER && !any) ok = false;
        }
        if (!ok) {
            *bad_event = e;
            return SIMINF_E_EVENT_INDEX;
        }
    }
    return SIMINF_OK;
}

bool same_matrix(const int32_t* a, const int32_t* b, size_t n) {
    return n == 0 || std::memcmp(a, b, sizeof(int32_t) * n) == 0;
}

int device_cus(const siminf_model* m) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, m->device) != hipSuccess) return 0;
    return cus;
}

// Wall-clock ticks one in-kernel wait may last (options.wait_ms, default 60 s),
// at the rate of the device's constant real-time counter.
uint64_t wait_ticks(const siminf_model* m) {
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, m->device) != hipSuccess || khz <= 0)
        khz = 100000;
    const int64_t ms = m->opt.wait_ms > 0 ? m->opt.wait_ms : 60000;
    return (uint64_t)khz * (uint64_t)ms;
}

// Heaviest nodes worth a whole wavefront each.  A wide node walks its
// steps several times faster than a node sharing its wavefront with 63
// others but occupies 64 lanes, so only nodes that would otherwise set the
// critical path qualify: expected work above 1/div of the heaviest node's and
// above the share of the whole run one lane would get if the work were
// spread evenly over 34,560 lanes (the measured throughput of the device in
// lane-steps per lane-step time).  Needs the binned (work-sorted) node order.
int default_wide(const siminf_model* m, const Group& g, int div = 16) {
    if (m->opt.lanes == 1 || g.n == 0 || m->opt.order == 1) return 0;
    if (m->opt.lanes == 64 && m->opt.wide > 0) return std::min(m->opt.wide, g.n);
    if (div <= 0) return 0;
    const int64_t top = g.work[0];
    long double total = 0;
    for (int64_t w : g.work) total += (long double)w;
    const long double cut = std::max((long double)top / (long double)div, total / 34560.0L);
    int nb = 0;
    while (nb < g.n && nb < 4096 && (long double)g.work[nb] > cut) ++nb;
    return nb;
}

// The first 1/div of the nodes after the nbig wide ones (none for div <= 0):
// in the binned order, the heaviest of them, candidates for a group of
// lanes each.
int default_group(const Group& g, int nbig, int div) {
    if (div <= 0 || nbig >= g.n) return 0;
    return (g.n - nbig + div - 1) / div;
}

// Kernel and launch shape of one group.  want_mode applies to groups with
// external transfers: 0 auto (dataflow if every node wavefront fits on the
// device at once, else grid barrier), 1 barrier, 2 dataflow.
// LDS a lane-queue workgroup of wpb wavefronts needs: the day-to-record
// table (nb + 1 ints, padded to 8 bytes), and per wavefront its recording
// slots, the slots' global data and its counters.
size_t lane_queue_lds(const siminf_model* m, const Group& g, int wpb) {
    const size_t table = (size_t)(m->nb + 2) / 2 * sizeof(uint64_t);
    const size_t slots = m->record == SIMINF_RECORD_SUMS ? (size_t)LQ_SLOTS * m->ntspan * g.shape.nc : 0;
    // per wavefront: recording slots, each slot's global data, four counters
    return table + (size_t)wpb * (slots + (size_t)LQ_SLOTS * g.shape.ngd + 4) * sizeof(uint64_t);
}

// Kernel and launch shape of one group.  want_mode applies to groups with
// external transfers: 0 auto (dataflow if every node wavefront fits on the
// device at once, else grid barrier), 1 barrier, 2 dataflow.  lq_chunk > 0
// (groups without external transfers): the lane-queue kernel with chunks of
// that many nodes; nbig, pack and ngrp are then ignored.
int configure(siminf_model* m, Group& g, int block, int nbig, int pipeline, int want_mode, int pack, int ngrp,
              int lq_chunk, int lq_batch = 16) {
    drop_graph(m);
    KParams& p = g.p;
    p.lane_queue = 0;
    g.lq_chunk = 0;
    if (lq_chunk > 0 && g.n_e2 == 0 && !p.coupled && !is_generated(g.model) && p.solver == 0) {
        const int cus = device_cus(m);
        if (cus <= 0) return SIMINF_E_DEVICE;
        if (block == 0) block = 256;
        const int wpb = block / WAVE;
        const size_t lds = lane_queue_lds(m, g, wpb);
        if (lds > (size_t)LQ_LDS_BYTES) return SIMINF_E_UNSUPPORTED;
        const int per_cu = max_blocks_per_cu(g.model, MODE_FREE, pipeline == 1 ? 1 : 0, false, block, lds, true);
        if (per_cu <= 0) return SIMINF_E_DEVICE;
        // chunks: consecutive nodes of one run, at most lq_chunk of them and,
        // past a wavefront's worth of nodes, at most 1/8 of one wavefront's
        // share of the expected work, so that the chunks a wavefront still
        // works on at the end of the run are short
        long double total = 0;
        for (int64_t w : g.work) total += (long double)w;
        const long double budget = total / ((long double)per_cu * cus * wpb * 8.0L);
        std::vector<int4> ch;
        for (int k = 0; k < g.n;) {
            int e = k + 1;
            long double w = (long double)g.work[k];
            while (e < g.n && e - k < lq_chunk && g.node_run[e] == g.node_run[k] &&
                   (e - k < WAVE || w + g.work[e] <= budget)) {
                w += (long double)g.work[e];
                ++e;
            }
            ch.push_back(make_int4(k, e, g.node_run[k], 0));
            k = e;
        }
        if ((int)ch.size() > g.chunk_cap) {
            // more pieces than the table holds: the table's size was set for
            // chunks of at least 64 nodes; grow it
            void* grown = nullptr;
            if (hipMalloc(&grown, sizeof(int4) * ch.size()) != hipSuccess) return SIMINF_E_ALLOC;
            m->owned.push_back(grown);
            g.d_chunks = (int4*)grown;
            g.chunk_cap = (int)ch.size();
        }
        if (!ch.empty() && hipMemcpy(g.d_chunks, ch.data(), sizeof(int4) * ch.size(), hipMemcpyHostToDevice) !=
                               hipSuccess)
            return SIMINF_E_DEVICE;
        int blocks = std::max(1, std::min(per_cu * cus, ((int)ch.size() + wpb - 1) / wpb));
        if (m->opt.max_blocks > 0) blocks = std::min(blocks, m->opt.max_blocks);
        g.mode = MODE_FREE;
        p.mode = MODE_FREE;
        p.lane_queue = 1;
        p.nlchunks = (int)ch.size();
        p.lchunks = g.d_chunks;
        p.pipeline = pipeline == 1 ? 1 : 0;
        p.nbig = 0;
        p.pack = WAVE;
        p.ngrp = 0;
        p.ngw = 0;
        p.nmajor = 0;
        p.nchunks = 0;
        g.block = block;
        g.blocks = blocks;
        g.shmem = lds;
        g.lq_chunk = lq_chunk;
        g.lq_batch = std::max(1, std::min(lq_batch, WAVE));
        p.lq_batch = g.lq_batch;
        p.nblocks = blocks;
        return SIMINF_OK;
    }
    if (lq_chunk > 0) return SIMINF_E_UNSUPPORTED;
    // a generated model, and the all events method, run one lane per node
    const bool aem = p.solver == 1;
    if (is_generated(g.model) || aem) {
        nbig = 0;
        ngrp = 0;
    }
    // the coupled post-time step: the dataflow kernel only, every node resident
    const bool coupled = p.coupled != 0;
    if (coupled && want_mode == 1) return SIMINF_E_UNSUPPORTED;
    const int n = g.n;
    const int cus = device_cus(m);
    if (cus <= 0) return SIMINF_E_DEVICE;
    nbig = std::max(0, std::min(nbig, n));
    // nodes on a group of lanes: only where the lattice walk applies
    const int per_grp = WAVE / GROUP_LANES;
    ngrp = p.lattice ? std::max(0, std::min(ngrp, n - nbig)) : 0;
    // pack 0 (auto): 64 nodes to a wavefront, unless that leaves CUs without a
    // wavefront; then the largest packing that gives every SIMD one (at least
    // 16 nodes to a wavefront in the coupled kernel, whose posts every
    // wavefront polls), else the smallest allowed
    const bool auto_pack = pack == 0;
    if (auto_pack) {
        const long long major = (long long)nbig + (ngrp + per_grp - 1) / per_grp;
        const long long rest = n - nbig - ngrp;
        pack = WAVE;
        if (major + (rest + WAVE - 1) / WAVE < cus) {
            const int smallest = p.coupled ? 16 : 4;
            while (pack > smallest && major + (rest + pack - 1) / pack < (long long)cus * 4) pack /= 2;
        }
    }
    if (pack != 4 && pack != 8 && pack != 16 && pack != 32) pack = WAVE;
    // pipelining pays where lanes are scarce (latency-bound runs); with many
    // waves per SIMD the extra, unused last draw of each node-day only costs
    const int simd_lanes = cus * 4 * WAVE;
    p.pipeline = pipeline == 1 ? 1 : pipeline == 2 ? 0 : (n <= simd_lanes ? 1 : 0);
    if (block == 0) block = g.n_e2 > 0 || coupled ? 64 : 256;
    const int wpb = block / WAVE;
    int mode = MODE_FREE, blocks = 0;
    size_t shmem = 0;
    if (g.n_e2 > 0 || coupled) {
        if (want_mode == 0 || want_mode == 2) {
            int nb = nbig;
            int ng = std::min(ngrp, n - nb);
            int per_cu = max_blocks_per_cu(g.model, MODE_FLOW, p.pipeline, ng > 0, block, 0, false, aem);
            auto need = [&](int k, int gn) {
                return (k + (gn + per_grp - 1) / per_grp + (n - k - gn + pack - 1) / pack + wpb - 1) / wpb;
            };
            // every wavefront must be resident: undo an automatic packing
            // first, then drop the groups, then halve the wide nodes
            while (auto_pack && pack < WAVE && per_cu > 0 && need(nb, ng) > per_cu * cus) pack *= 2;
            if (ng > 0 && (per_cu <= 0 || need(nb, ng) > per_cu * cus)) {
                ng = 0;
                per_cu = max_blocks_per_cu(g.model, MODE_FLOW, p.pipeline, false, block, 0, false, aem);
            }
            while (nb > 0 && per_cu > 0 && need(nb, ng) > per_cu * cus) nb /= 2;
            if (per_cu > 0 && need(nb, std::min(ng, n - nb)) <= per_cu * cus) {
                mode = MODE_FLOW;
                nbig = nb;
                ngrp = std::min(ng, n - nb);
                blocks = std::max(1, need(nb, ngrp));
            } else if (want_mode == 2 || coupled) {
                return SIMINF_E_UNSUPPORTED;
            }
        }
        if (mode != MODE_FLOW) {
            mode = MODE_BARRIER;
            shmem = 0;
            nbig = 0;
            ngrp = 0;
            pack = WAVE;  // the barrier kernel strides over nodes 64 to a wavefront
            const int per_cu = max_blocks_per_cu(g.model, MODE_BARRIER, p.pipeline, false, block, 0, false, aem);
            if (per_cu <= 0) return SIMINF_E_DEVICE;
            blocks = std::max(1, std::min(per_cu * cus, (n + block - 1) / block));
            if (m->opt.max_blocks > 0) blocks = std::min(blocks, m->opt.max_blocks);
        }
    } else {
        const int per_cu = max_blocks_per_cu(g.model, MODE_FREE, p.pipeline, ngrp > 0, block, 0, false, aem);
        if (per_cu <= 0) return SIMINF_E_DEVICE;
        const int chunks = nbig + (ngrp + per_grp - 1) / per_grp + (n - nbig - ngrp + pack - 1) / pack;
        blocks = std::max(1, std::min(per_cu * cus, (chunks + wpb - 1) / wpb));
        if (m->opt.max_blocks > 0) blocks = std::min(blocks, m->opt.max_blocks);
    }
    g.mode = mode;
    p.mode = mode;
    p.nbig = nbig;
    p.pack = pack;
    p.ngrp = ngrp;
    p.ngw = (ngrp + per_grp - 1) / per_grp;
    p.nmajor = nbig + ngrp;
    p.nchunks = nbig + p.ngw + (n - nbig - ngrp + pack - 1) / pack;
    g.block = block;
    g.blocks = blocks;
    g.shmem = shmem;
    p.nblocks = blocks;
    return SIMINF_OK;
}

int create_impl(const siminf_spec* specs, int nspecs, const int32_t* reps, const siminf_options* opt,
                siminf_model** out) {
    if (!out) return SIMINF_E_ARG;
    *out = nullptr;
    if (!specs || nspecs < 1) return SIMINF_E_ARG;
    siminf_model* m = new (std::nothrow) siminf_model();
    if (!m) return SIMINF_E_ALLOC;
    *out = m;
    if (opt) m->opt = *opt;
    if (m->opt.record != SIMINF_RECORD_FULL && m->opt.record != SIMINF_RECORD_SUMS) {
        set_create_error(m, SIMINF_E_ARG, -1, -1);
        return SIMINF_E_ARG;
    }
    if (m->opt.block != 0 && (m->opt.block % 64 != 0 || m->opt.block < 64 || m->opt.block > 256)) {
        set_create_error(m, SIMINF_E_ARG, -1, -1);
        return SIMINF_E_ARG;
    }
    if (m->opt.pipeline < 0 || m->opt.pipeline > 2 || m->opt.mode < 0 || m->opt.mode > 2 || m->opt.wait_ms < 0 ||
        m->opt.lattice < 0 || m->opt.lattice > 2 || m->opt.graph < 0 || m->opt.graph > 1 || m->opt.solver < 0 ||
        m->opt.solver > 1) {
        set_create_error(m, SIMINF_E_ARG, -1, -1);
        return SIMINF_E_ARG;
    }
    if ((m->opt.pack != 0 && m->opt.pack != 4 && m->opt.pack != 8 && m->opt.pack != 16 && m->opt.pack != 32 &&
         m->opt.pack != 64) ||
        m->opt.group < -1) {
        set_create_error(m, SIMINF_E_ARG, -1, -1);
        return SIMINF_E_ARG;
    }
    if (m->opt.lane_queue < 0 || m->opt.lane_queue > 2 ||
        (m->opt.chunk != 0 && (m->opt.chunk < 64 || m->opt.chunk > (1 << 20))) || m->opt.batch < 0 ||
        m->opt.batch > WAVE) {
        set_create_error(m, SIMINF_E_ARG, -1, -1);
        return SIMINF_E_ARG;
    }
    if (m->opt.lanes != 0 && m->opt.lanes != 1 && m->opt.lanes != 64) {
        set_create_error(m, SIMINF_E_UNSUPPORTED, -1, -1);
        return SIMINF_E_UNSUPPORTED;
    }
    if (hipGetDevice(&m->device) != hipSuccess) return hip_fail(m);
    m->record = m->opt.record;
    m->nspec = nspecs;

    // ---- validate every spec; shared tspan; one S/G/E/N per model ----------
    for (int s = 0; s < nspecs; ++s) {
        int64_t bad = -1;
        const int rc = validate_spec(specs[s], &bad);
        if (rc) {
            set_create_error(m, rc, bad, -1);
            return rc;
        }
        if (reps && reps[s] < 0) {
            set_create_error(m, SIMINF_E_ARG, -1, -1);
            return SIMINF_E_ARG;
        }
        if (specs[s].Ntspan != specs[0].Ntspan ||
            std::memcmp(specs[s].tspan, specs[0].tspan, sizeof(double) * specs[0].Ntspan) != 0) {
            set_create_error(m, SIMINF_E_ARG, -1, -1);
            return SIMINF_E_ARG;
        }
    }
    const siminf_spec& s0 = specs[0];
    m->ntspan = s0.Ntspan;
    m->t0 = s0.tspan[0];
    const double tend = s0.tspan[s0.Ntspan - 1];
    m->T1 = (int64_t)std::floor(m->t0) + 1;
    m->nb = tend > m->t0 ? (int)(std::ceil(tend) - std::floor(m->t0)) : 0;
    if ((uint32_t)m->nb >= MAX_STEPS) {
        set_create_error(m, SIMINF_E_UNSUPPORTED, -1, -1);
        return SIMINF_E_UNSUPPORTED;
    }
    m->rec_off.assign(m->nb + 1, 0);
    {
        int rec = 0;
        while (rec < m->ntspan && s0.tspan[rec] <= m->t0) ++rec;
        m->first_rec = rec;
        m->rec_off[0] = rec;
        for (int b = 0; b < m->nb; ++b) {
            const double T = (double)(m->T1 + b);
            while (rec < m->ntspan && s0.tspan[rec] <= T) ++rec;
            m->rec_off[b + 1] = rec;
        }
    }

    // ---- runs and model groups ---------------------------------------------
    std::vector<int> group_of_model(SIMINF_GEN_LAST + 1, -1);  // built-in and generated model ids
    std::vector<int> group_spec0;
    int64_t noff = 0, eoff = 0;
    for (int s = 0; s < nspecs; ++s) {
        const int model = specs[s].model;
        if (model < 0 || model > SIMINF_GEN_LAST) {
            set_create_error(m, SIMINF_E_UNSUPPORTED, -1, -1);
            return SIMINF_E_UNSUPPORTED;
        }
        if (group_of_model[model] < 0) {
            group_of_model[model] = (int)m->groups.size();
            Group g;
            g.model = model;
            shape_of(model, &g.shape);
            m->groups.push_back(g);
            group_spec0.push_back(s);
        } else {
            const siminf_spec& a = specs[group_spec0[group_of_model[model]]];
            const siminf_spec& b = specs[s];
            bool same = a.Ecols == b.Ecols && a.Ncols == b.Ncols &&
                        same_matrix(a.S, b.S, (size_t)a.Nc * a.Nt) && same_matrix(a.G, b.G, (size_t)a.Nt * a.Nt) &&
                        same_matrix(a.E, b.E, (size_t)a.Nc * a.Ecols) && same_matrix(a.N, b.N, (size_t)a.Nc * a.Ncols);
            if (!same) {
                set_create_error(m, SIMINF_E_ARG, -1, -1);
                return SIMINF_E_ARG;
            }
        }
        const int nrep = reps ? reps[s] : 1;
        for (int r = 0; r < nrep; ++r) {
            RunInfo ri{s, group_of_model[model], noff, specs[s].Nn, eoff};
            m->runs.push_back(ri);
            noff += specs[s].Nn;
            eoff += specs[s].Nev;
        }
        m->ncmax = std::max(m->ncmax, specs[s].Nc);
        m->nvmax = std::max(m->nvmax, specs[s].Nv);
    }
    m->R = (int)m->runs.size();
    m->total_nodes = noff;
    m->total_events = eoff;
    if ((uint64_t)noff >= MAX_ORDINAL || (uint64_t)eoff >= MAX_ORDINAL || m->R >= (1 << 24) ||
        m->groups.size() > (size_t)MAX_GROUPS) {
        set_create_error(m, SIMINF_E_UNSUPPORTED, -1, -1);
        return SIMINF_E_UNSUPPORTED;
    }
    bool any_e2 = false;
    for (int s = 0; s < nspecs; ++s)
        for (int e = 0; e < specs[s].Nev; ++e) any_e2 |= specs[s].ev_type[e] == SIMINF_EXTTRANS;
    bool any_coupled = false;
    for (int s = 0; s < nspecs; ++s) any_coupled |= specs[s].model == M_SISE_SP;
    if ((any_e2 || any_coupled) && m->groups.size() > 1) {
        set_create_error(m, SIMINF_E_ARG, -1, -1);
        return SIMINF_E_ARG;
    }

    // ---- shared device tables ------------------------------------------------
    int ngd_max = 0;
    for (int s = 0; s < nspecs; ++s) ngd_max = std::max(ngd_max, specs[s].Ngd);
    std::vector<double> gdata((size_t)nspecs * std::max(ngd_max, 1), 0.0);
    for (int s = 0; s < nspecs; ++s)
        for (int k = 0; k < specs[s].Ngd; ++k) gdata[(size_t)s * ngd_max + k] = specs[s].gdata[k];
    std::vector<int32_t> run_spec(m->R);
    for (int r = 0; r < m->R; ++r) run_spec[r] = m->runs[r].spec;
    double* d_gdata;
    int32_t *d_run_spec, *d_rec_off;
    if (to_device(m->owned, gdata, &d_gdata) || to_device(m->owned, run_spec, &d_run_spec) ||
        to_device(m->owned, m->rec_off, &d_rec_off))
        return hip_fail(m);
    if (alloc_device(m->owned, 1, &m->d_rp) || hipHostMalloc((void**)&m->h_rp, sizeof(RunParams)) != hipSuccess)
        return hip_fail(m);
    if (alloc_device(m->owned, 1, &m->d_ctrl) || hipMemset(m->d_ctrl, 0, sizeof(Ctrl)) != hipSuccess)
        return hip_fail(m);
    std::vector<int32_t> pos(std::max<int64_t>(m->total_nodes, 1), 0);

    if (m->record == SIMINF_RECORD_SUMS) {
        m->sums_len = (long long)m->R * m->ntspan * m->ncmax;
        std::vector<unsigned long long> init(m->sums_len, 0ull);
        for (int r = 0; r < m->R; ++r) {
            const siminf_spec& s = specs[m->runs[r].spec];
            for (int mm = 0; mm < m->first_rec; ++mm)
                for (int i = 0; i < s.Nn; ++i)
                    for (int c = 0; c < s.Nc; ++c)
                        init[((size_t)r * m->ntspan + mm) * m->ncmax + c] += (unsigned long long)s.u0[(size_t)i * s.Nc + c];
        }
        if (to_device(m->owned, init, &m->d_sums_init) || alloc_device(m->owned, m->sums_len, &m->d_sums))
            return hip_fail(m);
    }

    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, m->device) != hipSuccess)
        return hip_fail(m);

    // ---- per model group -------------------------------------------------------
    for (size_t gi = 0; gi < m->groups.size(); ++gi) {
        Group& g = m->groups[gi];
        const siminf_spec& sp = specs[group_spec0[gi]];
        const int nc = g.shape.nc, nv = g.shape.nv, nld = g.shape.nld;
        // nodes of this group, in input order, then binned
        struct NodeRef {
            int run;
            int32_t idx;
            int64_t work;
        };
        std::vector<NodeRef> nodes;
        std::vector<int> grp_runs;
        for (int r = 0; r < m->R; ++r)
            if (m->runs[r].group == (int)gi) grp_runs.push_back(r);
        // expected work of each node of each spec: the larger of its initial
        // and its mean population over the run, plus 8 per event it takes
        // part in.  The mean counts every scheduled change from the day after
        // it applies (a change given as a proportion is priced at the initial
        // population): transfers can make a node that starts small the
        // heaviest of all, while an epidemic in a large node is heaviest early.
        std::vector<std::vector<int64_t>> spec_work(nspecs);
        std::vector<std::vector<int32_t>> spec_order(nspecs);
        for (int r : grp_runs) {
            const int si = m->runs[r].spec;
            if (!spec_work[si].empty() || specs[si].Nn == 0) continue;
            const siminf_spec& s = specs[si];
            std::vector<int64_t>& w = spec_work[si];
            std::vector<double> pop(s.Nn, 0.0), popdays(s.Nn, 0.0);
            for (int i = 0; i < s.Nn; ++i)
                for (int c = 0; c < s.Nc; ++c) pop[i] += s.u0[(size_t)i * s.Nc + c];
            const double nbd = std::max(1, m->nb);
            for (int i = 0; i < s.Nn; ++i) popdays[i] = pop[i] * nbd;
            std::vector<int64_t> touches(s.Nn, 0);
            for (int e = 0; e < s.Nev; ++e) {
                const int ty = s.ev_type[e], src = s.ev_node[e];
                touches[src] += 1;
                if (ty == SIMINF_EXTTRANS) touches[s.ev_dest[e]] += 1;
                const int64_t step = std::max<int64_t>(0, (int64_t)s.ev_time[e] - m->T1);
                if (step >= m->nb || ty == SIMINF_INTTRANS) continue;
                const double days = nbd - 1.0 - (double)step;
                const double moved = s.ev_n[e] > 0 ? (double)s.ev_n[e] : s.ev_prop[e] * pop[src];
                if (ty == SIMINF_ENTER) {
                    popdays[src] += moved * days;
                } else {
                    popdays[src] -= moved * days;
                    if (ty == SIMINF_EXTTRANS) popdays[s.ev_dest[e]] += moved * days;
                }
            }
            w.assign(s.Nn, 0);
            for (int i = 0; i < s.Nn; ++i)
                w[i] = (int64_t)std::max(pop[i], popdays[i] / nbd) + 8 * touches[i];
            std::vector<int32_t>& o = spec_order[si];
            o.resize(s.Nn);
            std::iota(o.begin(), o.end(), 0);
            if (m->opt.order == 0)
                std::stable_sort(o.begin(), o.end(), [&](int32_t a, int32_t b) { return w[a] > w[b]; });
        }
        if (m->opt.order == 0 && grp_runs.size() > 1) {
            // batches: run-major, runs by their heaviest node (longest first on
            // the work queue), each run's nodes by expected work; a wavefront
            // then mostly holds nodes of one run with similar work
            std::vector<int> runs_sorted = grp_runs;
            auto top = [&](int r) {
                const int si = m->runs[r].spec;
                return spec_order[si].empty() ? (int64_t)0 : spec_work[si][spec_order[si][0]];
            };
            std::stable_sort(runs_sorted.begin(), runs_sorted.end(), [&](int a, int b) { return top(a) > top(b); });
            for (int r : runs_sorted) {
                const int si = m->runs[r].spec;
                for (int32_t i : spec_order[si]) nodes.push_back({r, i, spec_work[si][i]});
            }
        } else {
            for (int r : grp_runs) {
                const int si = m->runs[r].spec;
                for (int32_t i = 0; i < specs[si].Nn; ++i) nodes.push_back({r, i, spec_work[si][i]});
            }
            if (m->opt.order == 0)
                std::stable_sort(nodes.begin(), nodes.end(),
                                 [](const NodeRef& a, const NodeRef& b) { return a.work > b.work; });
        }
        const int n = (int)nodes.size();
        g.n = n;
        g.work.resize(n);
        for (int k = 0; k < n; ++k) g.work[k] = nodes[k].work;
        std::vector<int32_t> u0s((size_t)nc * n), node_run(n), node_idx(n);
        std::vector<double> v0s((size_t)nv * n), lds((size_t)nld * n);
        std::vector<int64_t> node_ord(n);
        for (int k = 0; k < n; ++k) {
            const NodeRef& nr = nodes[k];
            const siminf_spec& s = specs[m->runs[nr.run].spec];
            for (int c = 0; c < nc; ++c) u0s[(size_t)c * n + k] = s.u0[(size_t)nr.idx * nc + c];
            for (int c = 0; c < nv; ++c) v0s[(size_t)c * n + k] = s.v0[(size_t)nr.idx * nv + c];
            for (int l = 0; l < nld; ++l) lds[(size_t)l * n + k] = s.ldata[(size_t)nr.idx * s.Nld + l];
            node_run[k] = nr.run;
            node_idx[k] = nr.idx;
            node_ord[k] = m->runs[nr.run].noff + nr.idx;
            pos[m->runs[nr.run].noff + nr.idx] = k;
        }
        // spatial coupling: each node's neighbours at their internal positions
        // in stored order, with the weight D / d of each pair (one IEEE
        // division, as the model writes it), then the nodes that list it but
        // that it does not list (waited for only)
        std::vector<int32_t> cpl_off, cpl_fend, cpl_idx;
        std::vector<double> cpl_w;
        const bool coupled = g.model == M_SISE_SP;
        if (coupled) {
            std::vector<std::vector<int32_t>> readers(n);
            for (int k = 0; k < n; ++k) {
                const NodeRef& nr = nodes[k];
                const siminf_spec& sp2 = specs[m->runs[nr.run].spec];
                for (int e = sp2.nb_ptr[nr.idx]; e < sp2.nb_ptr[nr.idx + 1]; ++e)
                    readers[pos[m->runs[nr.run].noff + sp2.nb_idx[e]]].push_back(k);
            }
            cpl_off.assign(n + 1, 0);
            cpl_fend.assign(n, 0);
            std::vector<int32_t> fwd;
            for (int k = 0; k < n; ++k) {
                const NodeRef& nr = nodes[k];
                const siminf_spec& sp2 = specs[m->runs[nr.run].spec];
                fwd.clear();
                for (int e = sp2.nb_ptr[nr.idx]; e < sp2.nb_ptr[nr.idx + 1]; ++e) {
                    const int32_t j = pos[m->runs[nr.run].noff + sp2.nb_idx[e]];
                    cpl_idx.push_back(j);
                    cpl_w.push_back(sp2.gdata[7] / sp2.nb_dist[e]);
                    fwd.push_back(j);
                }
                cpl_fend[k] = (int32_t)cpl_idx.size();
                std::sort(fwd.begin(), fwd.end());
                std::vector<int32_t>& rd = readers[k];
                std::sort(rd.begin(), rd.end());
                rd.erase(std::unique(rd.begin(), rd.end()), rd.end());
                for (int32_t j : rd)
                    if (!std::binary_search(fwd.begin(), fwd.end(), j)) {
                        cpl_idx.push_back(j);
                        cpl_w.push_back(0.0);
                    }
                cpl_off[k + 1] = (int32_t)cpl_idx.size();
            }
        }
        // events: E1 in node-major CSR, E2 grouped by step and conflict level
        struct Ev {
            int run;
            int32_t e;
        };
        std::vector<Ev> e1, e2;
        for (int r : grp_runs) {
            const siminf_spec& s = specs[m->runs[r].spec];
            for (int e = 0; e < s.Nev; ++e)
                (s.ev_type[e] == SIMINF_EXTTRANS ? e2 : e1).push_back({r, e});
        }
        auto local = [&](int run, int32_t i) { return pos[m->runs[run].noff + i]; };
        auto S_of = [&](int run) -> const siminf_spec& { return specs[m->runs[run].spec]; };
        std::stable_sort(e1.begin(), e1.end(), [&](const Ev& a, const Ev& b) {
            const siminf_spec &sa = S_of(a.run), &sb = S_of(b.run);
            const int ka = local(a.run, sa.ev_node[a.e]), kb = local(b.run, sb.ev_node[b.e]);
            return std::make_tuple(ka, sa.ev_time[a.e], sa.ev_type[a.e], a.e) <
                   std::make_tuple(kb, sb.ev_time[b.e], sb.ev_type[b.e], b.e);
        });
        std::vector<int32_t> e1_off(n + 1, 0);
        for (const Ev& x : e1) e1_off[local(x.run, S_of(x.run).ev_node[x.e]) + 1] += 1;
        for (int k = 0; k < n; ++k) e1_off[k + 1] += e1_off[k];
        // step of an external transfer: first boundary T >= its time
        auto step_of = [&](const Ev& x) -> int64_t {
            const int64_t t = S_of(x.run).ev_time[x.e];
            return std::max<int64_t>(0, t - m->T1);
        };
        std::vector<Ev> e2k;
        for (const Ev& x : e2)
            if (step_of(x) < m->nb) e2k.push_back(x);
        std::stable_sort(e2k.begin(), e2k.end(), [&](const Ev& a, const Ev& b) {
            return std::make_tuple(step_of(a), S_of(a.run).ev_time[a.e], a.run, a.e) <
                   std::make_tuple(step_of(b), S_of(b.run).ev_time[b.e], b.run, b.e);
        });
        // conflict levels: an event's level is one more than the latest level of
        // any earlier same-step event touching its source or destination node
        std::vector<int32_t> lvl(e2k.size(), 0), last(n, -1);
        std::vector<int32_t> touched;
        std::vector<int32_t> e2_step(m->nb + 1, 0);
        std::vector<int32_t> e2_lvl;
        std::vector<size_t> order2;
        {
            size_t a = 0;
            int32_t level_base = 0;
            for (int b = 0; b < m->nb; ++b) {
                e2_step[b] = level_base;
                size_t z = a;
                int depth = 0;
                while (z < e2k.size() && step_of(e2k[z]) == b) {
                    const siminf_spec& s = S_of(e2k[z].run);
                    const int src = local(e2k[z].run, s.ev_node[e2k[z].e]);
                    const int dst = local(e2k[z].run, s.ev_dest[e2k[z].e]);
                    const int L = std::max(last[src], last[dst]) + 1;
                    lvl[z] = L;
                    last[src] = last[dst] = L;
                    touched.push_back(src);
                    touched.push_back(dst);
                    depth = std::max(depth, L + 1);
                    ++z;
                }
                std::vector<size_t> idx(z - a);
                std::iota(idx.begin(), idx.end(), a);
                std::stable_sort(idx.begin(), idx.end(), [&](size_t x, size_t y) { return lvl[x] < lvl[y]; });
                size_t c = 0;
                for (int L = 0; L < depth; ++L) {
                    e2_lvl.push_back((int32_t)order2.size());
                    while (c < idx.size() && lvl[idx[c]] == L) order2.push_back(idx[c++]);
                }
                level_base += depth;
                for (int t : touched) last[t] = -1;
                touched.clear();
                a = z;
            }
            e2_step[m->nb] = level_base;
            e2_lvl.push_back((int32_t)order2.size());
        }
        g.n_e1 = (int64_t)e1.size();
        g.n_e2 = (int64_t)order2.size();
        g.n_levels = (int64_t)e2_lvl.size() - 1;

        // per-node lists of external transfers in key order, for the dataflow
        // kernel: the source samples, the destination receives (a transfer from
        // a node to itself is one item with both roles)
        std::vector<int32_t> e2n_off(n + 1, 0);
        std::vector<int4> e2n_item;
        std::vector<size_t> e2n_src;  // index into order2 of each item (for its record)
        {
            std::vector<std::vector<std::pair<int4, size_t>>> per(n);
            size_t j = 0;
            for (int b = 0; b < m->nb; ++b) {
                const size_t jend = (size_t)e2_lvl[e2_step[b + 1]];
                for (; j < jend; ++j) {
                    const Ev& x = e2k[order2[j]];
                    const siminf_spec& s = S_of(x.run);
                    const int src = local(x.run, s.ev_node[x.e]);
                    const int dst = local(x.run, s.ev_dest[x.e]);
                    per[src].push_back({make_int4((int)j, b, src == dst ? 2 : 0, x.run), j});
                    if (dst != src) per[dst].push_back({make_int4((int)j, b, 1, x.run), j});
                }
            }
            // within a node, the items must follow the serial (key) order, which
            // the level order of a step does not keep: sort by the event's key
            for (int k = 0; k < n; ++k) {
                std::stable_sort(per[k].begin(), per[k].end(), [&](const auto& A, const auto& B) {
                    const Ev& xa = e2k[order2[A.second]];
                    const Ev& xb = e2k[order2[B.second]];
                    return std::make_tuple(A.first.y, S_of(xa.run).ev_time[xa.e], xa.run, xa.e) <
                           std::make_tuple(B.first.y, S_of(xb.run).ev_time[xb.e], xb.run, xb.e);
                });
                e2n_off[k + 1] = e2n_off[k] + (int32_t)per[k].size();
                for (auto& it : per[k]) {
                    e2n_item.push_back(it.first);
                    e2n_src.push_back(it.second);
                }
            }
        }

        // packed event records (select mask and shift targets resolved here)
        std::vector<int4> e2_rec_host;
        auto fill = [&](const std::vector<Ev>& list, const std::vector<size_t>* perm, EventSoA* soa,
                        bool transfers) -> bool {
            const size_t cnt = perm ? perm->size() : list.size();
            std::vector<int4> rec(cnt);
            std::vector<int32_t> nd(transfers ? cnt : 0), ds(transfers ? cnt : 0), rn(transfers ? cnt : 0);
            std::vector<double> prop(cnt);
            std::vector<int64_t> ord(cnt);
            for (size_t j = 0; j < cnt; ++j) {
                const Ev& x = perm ? list[(*perm)[j]] : list[j];
                const siminf_spec& s = S_of(x.run);
                const int sel = s.ev_select[x.e], q = s.ev_shift[x.e];
                if (is_generated(g.model)) {
                    // a generated model's tables are compiled in: the word
                    // names the column of E and the column of N plus one
                    const int qq = (q >= 0 && s.ev_type[x.e] != SIMINF_ENTER) ? q + 1 : 0;
                    const uint32_t wd = (uint32_t)s.ev_type[x.e] | ((uint32_t)sel << 2) | ((uint32_t)qq << 12);
                    rec[j] = make_int4(s.ev_time[x.e], (int32_t)wd, s.ev_n[x.e], x.e);
                    prop[j] = s.ev_prop[x.e];
                    ord[j] = m->runs[x.run].eoff + x.e;
                    if (transfers) {
                        nd[j] = local(x.run, s.ev_node[x.e]);
                        ds[j] = local(x.run, s.ev_dest[x.e]);
                        rn[j] = x.run;
                    }
                    continue;
                }
                uint32_t mask = 0;
                int target[MAX_NC] = {0, 1, 2, 3};
                for (int c = 0; c < nc; ++c) {
                    if (s.E[(size_t)sel * nc + c]) mask |= 1u << c;
                    if (q >= 0 && s.ev_type[x.e] != SIMINF_ENTER) target[c] = c + s.N[(size_t)q * nc + c];
                    if (target[c] < 0 || target[c] >= nc) target[c] = c;  // unselected rows are never used
                }
                rec[j] = make_int4(s.ev_time[x.e], pack_event(s.ev_type[x.e], mask, target, nc), s.ev_n[x.e], x.e);
                prop[j] = s.ev_prop[x.e];
                ord[j] = m->runs[x.run].eoff + x.e;
                if (transfers) {
                    nd[j] = local(x.run, s.ev_node[x.e]);
                    ds[j] = local(x.run, s.ev_dest[x.e]);
                    rn[j] = x.run;
                }
            }
            int4* a_rec;
            double* a_prop;
            int64_t* a_ord;
            int32_t *a_nd = nullptr, *a_ds = nullptr, *a_rn = nullptr;
            if (to_device(m->owned, rec, &a_rec) || to_device(m->owned, prop, &a_prop) ||
                to_device(m->owned, ord, &a_ord))
                return false;
            if (transfers && (to_device(m->owned, nd, &a_nd) || to_device(m->owned, ds, &a_ds) ||
                              to_device(m->owned, rn, &a_rn)))
                return false;
            *soa = EventSoA{a_rec, a_prop, a_ord, a_nd, a_ds, a_rn};
            if (transfers) e2_rec_host = rec;
            return true;
        };
        KParams& p = g.p;
        p = KParams{};
        p.wait_ticks = wait_ticks(m);
        p.n = n;
        p.nb = m->nb;
        p.ntspan = m->ntspan;
        p.T1 = m->T1;
        p.t0 = m->t0;
        p.ngd = std::max(ngd_max, 1);
        for (int j = 0; j < (is_generated(g.model) ? 0 : g.shape.nt); ++j) {
            for (int c = 0; c < nc; ++c) p.S[c + j * nc] = sp.S[c + (size_t)j * nc];
            uint32_t mask = 0;
            for (int k = 0; k < g.shape.nt; ++k)
                if (sp.G[k + (size_t)j * g.shape.nt]) mask |= 1u << k;
            p.Gmask[j] = mask;
        }
        p.lattice = !is_generated(g.model) && m->opt.lattice != 2 && g.shape.nt == 2 && p.Gmask[0] == 3u &&
                            p.Gmask[1] == 3u
                        ? 1
                        : 0;
        int32_t *d_u0, *d_nrun, *d_nidx, *d_e1off, *d_e2step, *d_e2lvl, *d_e2noff;
        double *d_v0, *d_ld;
        int64_t* d_nord;
        if (to_device(m->owned, u0s, &d_u0) || to_device(m->owned, v0s, &d_v0) || to_device(m->owned, lds, &d_ld) ||
            to_device(m->owned, node_run, &d_nrun) || to_device(m->owned, node_idx, &d_nidx) ||
            to_device(m->owned, node_ord, &d_nord) || to_device(m->owned, e1_off, &d_e1off) ||
            to_device(m->owned, e2_step, &d_e2step) || to_device(m->owned, e2_lvl, &d_e2lvl) ||
            to_device(m->owned, e2n_off, &d_e2noff))
            return hip_fail(m);
        if (!fill(e1, nullptr, &p.e1, false) || !fill(e2k, &order2, &p.e2, true)) return hip_fail(m);
        {
            std::vector<int4> e2n_rec(e2n_item.size());
            for (size_t i = 0; i < e2n_item.size(); ++i) e2n_rec[i] = e2_rec_host[e2n_src[i]];
            int4 *d_item, *d_nrec;
            if (to_device(m->owned, e2n_item, &d_item) || to_device(m->owned, e2n_rec, &d_nrec)) return hip_fail(m);
            p.e2n_item = d_item;
            p.e2n_rec = d_nrec;
        }
        p.rec_off = d_rec_off;
        p.u0 = d_u0;
        p.v0 = d_v0;
        p.ld = d_ld;
        p.node_run = d_nrun;
        p.node_idx = d_nidx;
        p.node_ord = d_nord;
        p.gdata = d_gdata;
        p.run_spec = d_run_spec;
        p.e1_off = d_e1off;
        p.e2_step = d_e2step;
        p.e2_lvl = d_e2lvl;
        p.e2n_off = d_e2noff;
        p.n_e2 = (int32_t)order2.size();
        p.record = m->record;
        p.sums_nc = m->ncmax;
        p.sums = m->d_sums;
        if (m->record == SIMINF_RECORD_FULL) {
            if (alloc_device(m->owned, (size_t)m->ntspan * nc * n, &p.U) ||
                alloc_device(m->owned, (size_t)m->ntspan * std::max(nv, 1) * n, &p.V))
                return hip_fail(m);
        }
        p.ctrl = m->d_ctrl;
        p.rp = m->d_rp;
        p.group = (int)gi;
        p.solver = m->opt.solver;
        p.nt = g.shape.nt;
        if (p.solver == 1 &&
            (alloc_device(m->owned, (size_t)p.nt * n, &p.aem_T) || alloc_device(m->owned, (size_t)p.nt * n, &p.aem_P) ||
             alloc_device(m->owned, (size_t)p.nt * n, &p.aem_K)))
            return hip_fail(m);
        p.coupled = coupled ? 1 : 0;
        if (coupled) {
            int32_t *d_coff, *d_cfend, *d_cidx;
            double* d_cw;
            if (to_device(m->owned, cpl_off, &d_coff) || to_device(m->owned, cpl_fend, &d_cfend) ||
                to_device(m->owned, cpl_idx, &d_cidx) || to_device(m->owned, cpl_w, &d_cw) ||
                alloc_device(m->owned, (size_t)2 * n, &p.cpl_post))
                return hip_fail(m);
            p.cpl_off = d_coff;
            p.cpl_fend = d_cfend;
            p.cpl_idx = d_cidx;
            p.cpl_w = d_cw;
        }
        if (g.n_e2 > 0) {
            // live state for the transfer kernels (both variants)
            if (alloc_device(m->owned, (size_t)nc * n, &p.u) || alloc_device(m->owned, (size_t)std::max(nv, 1) * n, &p.v) ||
                alloc_device(m->owned, (size_t)n, &p.e1_cur) || alloc_device(m->owned, (size_t)p.n_e2, &p.mail) ||
                alloc_device(m->owned, (size_t)p.n_e2 * nc, &p.mail_big))
                return hip_fail(m);
        }
        g.node_run = node_run;
        int lq = 0;
        if (g.n_e2 == 0 && !coupled && !is_generated(g.model) && m->opt.solver == 0) {
            // the lane-queue chunk table: at most one chunk per run and per 64 nodes more
            g.chunk_cap = (int)grp_runs.size() + n / 64 + 1;
            if (alloc_device(m->owned, (size_t)g.chunk_cap, &g.d_chunks)) return hip_fail(m);
            const int chunk = m->opt.chunk > 0 ? m->opt.chunk : 512;
            const bool shaped = m->opt.lanes != 0 || m->opt.wide != 0 || m->opt.group != 0 || m->opt.pack != 0;
            const int wpb = (m->opt.block ? m->opt.block : 256) / WAVE;
            if (m->opt.lane_queue == 1)
                lq = chunk;
            else if (m->opt.lane_queue == 0 && !shaped && (int64_t)n >= (int64_t)cus * 4 * WAVE &&
                     lane_queue_lds(m, g, wpb) <= (size_t)LQ_LDS_BYTES)
                lq = chunk;
        } else if (m->opt.lane_queue == 1) {
            set_create_error(m, SIMINF_E_UNSUPPORTED, -1, -1);
            return SIMINF_E_UNSUPPORTED;
        }
        const int nb = default_wide(m, g);
        const int rc = configure(m, g, m->opt.block, nb, m->opt.pipeline, m->opt.mode, m->opt.pack,
                                 m->opt.group < 0 ? g.n : m->opt.group, lq, m->opt.batch ? m->opt.batch : 16);
        if (rc) {
            set_create_error(m, rc, -1, -1);
            return rc;
        }
    }
    if (to_device(m->owned, pos, &m->d_pos)) return hip_fail(m);
    for (hipEvent_t& e : m->ev)
        if (hipEventCreate(&e) != hipSuccess) return hip_fail(m);
    if (m->groups.size() > 1) {
        if (hipEventCreateWithFlags(&m->fork, hipEventDisableTiming) != hipSuccess) return hip_fail(m);
        for (size_t gi = 1; gi < m->groups.size(); ++gi) {
            hipStream_t ss = nullptr;
            hipEvent_t je = nullptr;
            if (hipStreamCreateWithFlags(&ss, hipStreamNonBlocking) != hipSuccess) return hip_fail(m);
            m->side.push_back(ss);
            if (hipEventCreateWithFlags(&je, hipEventDisableTiming) != hipSuccess) return hip_fail(m);
            m->joins.push_back(je);
        }
    }
    return SIMINF_OK;
}

void decode_error(siminf_model* m, uint64_t key) {
    m->err_code = -(int32_t)(key & 0xF);
    m->err_step = (int64_t)(key >> 44);
    m->err_phase = (int32_t)((key >> 42) & 3);
    const int64_t ord = (int64_t)((key >> 4) & ((1ull << 38) - 1));
    const bool node_phase = m->err_phase == PH_SSA || m->err_phase == PH_PTS;
    int lo = 0, hi = m->R - 1, run = 0;
    while (lo <= hi) {
        const int mid = (lo + hi) / 2;
        const int64_t off = node_phase ? m->runs[mid].noff : m->runs[mid].eoff;
        if (off <= ord) {
            run = mid;
            lo = mid + 1;
        } else {
            hi = mid - 1;
        }
    }
    // skip empty runs that share the same offset
    if (node_phase)
        while (run + 1 < m->R && m->runs[run + 1].noff <= ord && m->runs[run].nn == 0) ++run;
    m->err_run = run;
    m->err_index = ord - (node_phase ? m->runs[run].noff : m->runs[run].eoff);
}

int finish(siminf_model* m) {
    if (!m->pending) return m->status;
    m->pending = false;
    if (hipStreamSynchronize(m->last_stream) != hipSuccess) return hip_fail(m);
    Ctrl c;
    if (hipMemcpy(&c, m->d_ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost) != hipSuccess) return hip_fail(m);
    for (int i = 0; i < 4; ++i) m->counters[i] = c.counters[i];
    m->err_code = 0;
    m->err_step = -1;
    m->err_phase = -1;
    m->err_index = -1;
    m->err_run = -1;
    if (c.abort) {
        m->err_code = SIMINF_E_DEVICE;
        m->status = SIMINF_E_DEVICE;
        return m->status;
    }
    if (c.err_key != NO_ERROR) decode_error(m, c.err_key);
    m->status = m->err_code;
    return m->status;
}

}  // namespace

extern "C" {

int siminf_create(const siminf_spec* spec, const siminf_options* opt, siminf_model** out) {
    return create_impl(spec, 1, nullptr, opt, out);
}

int siminf_create_batch(const siminf_spec* specs, int32_t nspecs, const int32_t* replicates,
                        const siminf_options* opt, siminf_model** out) {
    return create_impl(specs, nspecs, replicates, opt, out);
}

namespace {

// The launches of one run after its parameters are in place: the init
// kernel(s), then (mark recorded on the stream between them if given) one
// SSA kernel per group.
int enqueue_launches(siminf_model* m, hipStream_t st, hipEvent_t mark = nullptr) {
    for (size_t gi = 0; gi < m->groups.size(); ++gi) {
        Group& g = m->groups[gi];
        if (launch_init(g.p, g.shape.nc, g.shape.nv, m->first_rec, gi == 0,
                        gi == 0 ? m->d_sums_init : nullptr, gi == 0 ? m->sums_len : 0, st) != hipSuccess)
            return SIMINF_E_DEVICE;
    }
    if (m->groups.empty()) {
        KParams p{};
        p.ctrl = m->d_ctrl;
        p.sums = m->d_sums;
        p.rp = m->d_rp;
        if (launch_init(p, 0, 0, 0, true, m->d_sums_init, m->sums_len, st) != hipSuccess) return SIMINF_E_DEVICE;
    }
    if (mark && hipEventRecord(mark, st) != hipSuccess) return SIMINF_E_DEVICE;
    // the first non-empty group on the run's stream, every other one on a
    // side stream that waits for the initialisation and is waited for
    std::vector<size_t> busy;
    for (size_t gi = 0; gi < m->groups.size(); ++gi)
        if (m->groups[gi].n > 0) busy.push_back(gi);
    if (busy.size() > 1 && hipEventRecord(m->fork, st) != hipSuccess) return SIMINF_E_DEVICE;
    for (size_t j = 1; j < busy.size(); ++j) {
        const Group& g = m->groups[busy[j]];
        hipStream_t ss = m->side[j - 1];
        if (hipStreamWaitEvent(ss, m->fork, 0) != hipSuccess ||
            launch_group(g.model, g.p, g.block, g.blocks, g.shmem, ss) != hipSuccess ||
            hipEventRecord(m->joins[j - 1], ss) != hipSuccess)
            return SIMINF_E_DEVICE;
    }
    if (!busy.empty()) {
        const Group& g = m->groups[busy[0]];
        if (launch_group(g.model, g.p, g.block, g.blocks, g.shmem, st) != hipSuccess) return SIMINF_E_DEVICE;
    }
    for (size_t j = 1; j < busy.size(); ++j)
        if (hipStreamWaitEvent(st, m->joins[j - 1], 0) != hipSuccess) return SIMINF_E_DEVICE;
    return SIMINF_OK;
}

// Captures enqueue_launches on a private stream into an executable graph.
int capture_graph(siminf_model* m) {
    for (const Group& g : m->groups)
        if (g.n > 0 && g.p.mode != MODE_FREE) return SIMINF_E_UNSUPPORTED;  // cooperative launches
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return SIMINF_E_DEVICE;
    int rc = SIMINF_OK;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        rc = SIMINF_E_DEVICE;
    } else {
        rc = enqueue_launches(m, cs);
        hipGraph_t graph = nullptr;
        if (hipStreamEndCapture(cs, &graph) != hipSuccess || !graph) {
            rc = SIMINF_E_DEVICE;
        } else if (rc == SIMINF_OK && hipGraphInstantiate(&m->gexec, graph, nullptr, nullptr, 0) != hipSuccess) {
            m->gexec = nullptr;
            rc = SIMINF_E_DEVICE;
        }
        m->graph = graph;
    }
    (void)hipStreamDestroy(cs);
    if (rc != SIMINF_OK) drop_graph(m);
    return rc;
}

}  // namespace

int siminf_run(siminf_model* m, uint64_t seed, uint32_t stream_base, void* hip_stream) {
    if (!m) return SIMINF_E_ARG;
    if ((uint64_t)stream_base + (uint64_t)m->R > (1ull << 24)) return SIMINF_E_ARG;
    if (m->pending) finish(m);  // the staging buffer and the device state are free again
    hipStream_t st = (hipStream_t)hip_stream;
    if (m->opt.graph && !m->gexec) {
        const int rc = capture_graph(m);
        if (rc != SIMINF_OK) {
            m->status = rc;
            return rc;
        }
    }
    m->h_rp->seed = seed;
    m->h_rp->stream_base = stream_base;
    m->h_rp->pad = 0;
    if (hipEventRecord(m->ev[0], st) != hipSuccess ||
        hipMemcpyAsync(m->d_rp, m->h_rp, sizeof(RunParams), hipMemcpyHostToDevice, st) != hipSuccess)
        return hip_fail(m);
    if (m->gexec) {
        // the graph holds the init kernels too: timed with the SSA kernels
        if (hipEventRecord(m->ev[1], st) != hipSuccess || hipGraphLaunch(m->gexec, st) != hipSuccess)
            return hip_fail(m);
    } else if (enqueue_launches(m, st, m->ev[1]) != SIMINF_OK) {
        return hip_fail(m);
    }
    if (hipEventRecord(m->ev[2], st) != hipSuccess) return hip_fail(m);
    m->last_stream = st;
    m->pending = true;
    m->ran = true;
    m->status = 0;
    return SIMINF_OK;
}

int siminf_wait(siminf_model* m) {
    if (!m) return SIMINF_E_ARG;
    return finish(m);
}

int siminf_trajectory(siminf_model* m, int32_t run, int32_t* U, double* V, int32_t dst_is_device) {
    if (!m || run < 0 || run >= m->R) return SIMINF_E_ARG;
    if (m->record != SIMINF_RECORD_FULL) return SIMINF_E_ARG;
    if (!m->ran) return SIMINF_E_ARG;
    const int status = finish(m);
    if (status == SIMINF_E_DEVICE) return status;
    const RunInfo& ri = m->runs[run];
    const Group& g = m->groups[ri.group];
    const int nc = g.shape.nc, nv = g.shape.nv;
    const size_t nU = (size_t)m->ntspan * ri.nn * nc, nV = (size_t)m->ntspan * ri.nn * nv;
    if (ri.nn == 0) return status;
    int32_t* dU = nullptr;
    double* dV = nullptr;
    if (!dst_is_device) {
        // one staging buffer per handle, grown to the largest request
        const size_t need = sizeof(int32_t) * (U ? nU : 0) + sizeof(double) * ((V && nv > 0) ? nV : 0) + 16;
        if (need > m->stage_bytes) {
            if (m->stage) (void)hipFree(m->stage);
            m->stage = nullptr;
            m->stage_bytes = 0;
            if (hipMalloc(&m->stage, need) != hipSuccess) return SIMINF_E_ALLOC;
            m->stage_bytes = need;
        }
        char* base = (char*)m->stage;
        dV = (V && nv > 0) ? (double*)base : nullptr;
        dU = U ? (int32_t*)(base + ((V && nv > 0) ? sizeof(double) * nV : 0)) : nullptr;
    } else {
        dU = U;
        dV = nv > 0 ? V : nullptr;
    }
    hipStream_t st = m->last_stream;
    if (launch_gather(nc, nv, g.p.U, g.p.V, g.n, m->ntspan, g.p.nmajor, m->d_pos + ri.noff, ri.nn, dU, dV, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return SIMINF_E_DEVICE;
    if (!dst_is_device) {
        if (U && hipMemcpy(U, dU, sizeof(int32_t) * nU, hipMemcpyDeviceToHost) != hipSuccess) return SIMINF_E_DEVICE;
        if (dV && hipMemcpy(V, dV, sizeof(double) * nV, hipMemcpyDeviceToHost) != hipSuccess) return SIMINF_E_DEVICE;
    }
    return status;
}

int siminf_trajectory_sparse(siminf_model* m, int32_t run, int32_t which, int64_t nnz, const int64_t* col_ptr,
                             const int32_t* row_idx, double* values, int32_t dst_is_device) {
    if (!m || run < 0 || run >= m->R || (which != 0 && which != 1) || nnz < 0 || !col_ptr ||
        (nnz > 0 && (!row_idx || !values)))
        return SIMINF_E_ARG;
    if (m->record != SIMINF_RECORD_FULL || !m->ran) return SIMINF_E_ARG;
    const RunInfo& ri = m->runs[run];
    const Group& g = m->groups[ri.group];
    const int width = which == 0 ? g.shape.nc : g.shape.nv;
    const int64_t rows = (int64_t)ri.nn * width;
    // the pattern: nondecreasing column pointers from 0 to nnz, rows in range
    if (col_ptr[0] != 0 || col_ptr[m->ntspan] != nnz) return SIMINF_E_ARG;
    for (int k = 0; k < m->ntspan; ++k)
        if (col_ptr[k + 1] < col_ptr[k]) return SIMINF_E_ARG;
    for (int64_t e = 0; e < nnz; ++e)
        if (row_idx[e] < 0 || row_idx[e] >= rows) return SIMINF_E_ARG;
    const int status = finish(m);
    if (status == SIMINF_E_DEVICE) return status;
    if (nnz == 0) return status;
    // pattern and values through one device allocation of this call
    const size_t b_ptr = sizeof(int64_t) * ((size_t)m->ntspan + 1), b_idx = sizeof(int32_t) * (size_t)nnz;
    const size_t b_out = dst_is_device ? 0 : sizeof(double) * (size_t)nnz;
    const size_t off_idx = (b_ptr + 255) & ~(size_t)255, off_out = (off_idx + b_idx + 255) & ~(size_t)255;
    char* buf = nullptr;
    if (hipMalloc((void**)&buf, off_out + b_out) != hipSuccess) return SIMINF_E_ALLOC;
    double* out = dst_is_device ? values : (double*)(buf + off_out);
    hipStream_t st = m->last_stream;
    int rc = status;
    if (hipMemcpy(buf, col_ptr, b_ptr, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(buf + off_idx, row_idx, b_idx, hipMemcpyHostToDevice) != hipSuccess ||
        launch_sparse_gather(which == 0 ? g.p.U : nullptr, which == 0 ? nullptr : g.p.V, width, g.n, m->ntspan,
                             g.p.nmajor, m->d_pos + ri.noff, (const int64_t*)buf, (const int32_t*)(buf + off_idx),
                             nnz, out, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess ||
        (!dst_is_device && hipMemcpy(values, out, b_out, hipMemcpyDeviceToHost) != hipSuccess))
        rc = SIMINF_E_DEVICE;
    (void)hipFree(buf);
    return rc;
}

int siminf_sums(siminf_model* m, int64_t* sums, int32_t dst_is_device) {
    if (!m || !sums || m->record != SIMINF_RECORD_SUMS || !m->ran) return SIMINF_E_ARG;
    const int status = finish(m);
    if (status == SIMINF_E_DEVICE) return status;
    const size_t bytes = sizeof(int64_t) * (size_t)m->sums_len;
    if (bytes == 0) return status;
    if (hipMemcpy(sums, m->d_sums, bytes, dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost) !=
        hipSuccess)
        return SIMINF_E_DEVICE;
    return status;
}

int siminf_counters(siminf_model* m, uint64_t out[4]) {
    if (!m || !out) return SIMINF_E_ARG;
    finish(m);
    for (int i = 0; i < 4; ++i) out[i] = m->counters[i];
    return SIMINF_OK;
}

int siminf_shape(const siminf_model* m, int64_t out[6]) {
    if (!m || !out) return SIMINF_E_ARG;
    out[0] = m->R;
    out[1] = m->total_nodes;
    out[2] = m->ntspan;
    out[3] = m->ncmax;
    out[4] = m->nvmax;
    out[5] = m->nb;
    return SIMINF_OK;
}

int siminf_error_info(const siminf_model* m, int32_t* code, int64_t* step, int32_t* phase, int64_t* index,
                      int32_t* run) {
    if (!m) return SIMINF_E_ARG;
    if (code) *code = m->err_code;
    if (step) *step = m->err_step;
    if (phase) *phase = m->err_phase;
    if (index) *index = m->err_index;
    if (run) *run = m->err_run;
    return SIMINF_OK;
}

int siminf_error_message(const siminf_model* m, char* buf, size_t cap) {
    if (!m || !buf || cap == 0) return SIMINF_E_ARG;
    static const char* const phases[] = {"the SSA", "a node-local event", "an external transfer",
                                         "the post-time step"};
    const char* what = "";
    switch (m->err_code) {
        case SIMINF_E_NEG_STATE: what = "a transition made a compartment negative"; break;
        case SIMINF_E_BAD_RATE: what = "a transition rate was negative or not finite"; break;
        case SIMINF_E_EVENT_OVERDRAW: what = "an event asked for more individuals than the selected compartments hold"; break;
        case SIMINF_E_EVENT_INDEX: what = "an event names a node, select column or shift out of range"; break;
        case SIMINF_E_PTS: what = "the post-time-step function produced a non-finite state"; break;
        case SIMINF_E_STEP_LIMIT: what = "a node needed more than 2^24 SSA draws in one unit of time"; break;
        case SIMINF_E_DEVICE: what = "a HIP runtime error, or a wait inside a kernel passed its time limit"; break;
        case SIMINF_E_ARG: what = "an invalid argument or model"; break;
        case SIMINF_E_UNSUPPORTED: what = "a model or size the library does not implement"; break;
        case SIMINF_E_ALLOC: what = "an allocation failed"; break;
        default: break;
    }
    int n;
    if (m->err_code == 0) {
        n = std::snprintf(buf, cap, "SIMINF_OK");
    } else if (m->err_phase >= 0 && m->err_phase <= 3) {
        const bool node_phase = m->err_phase == PH_SSA || m->err_phase == PH_PTS;
        n = std::snprintf(buf, cap, "%s at day step %lld in %s, %s %lld of run %d: %s",
                          siminf_status_string(m->err_code), (long long)m->err_step, phases[m->err_phase],
                          node_phase ? "node" : "event", (long long)m->err_index, m->err_run, what);
    } else if (m->err_index >= 0) {
        n = std::snprintf(buf, cap, "%s at create, event %lld: %s", siminf_status_string(m->err_code),
                          (long long)m->err_index, what);
    } else {
        n = std::snprintf(buf, cap, "%s: %s", siminf_status_string(m->err_code), what);
    }
    return n < 0 ? SIMINF_E_ARG : SIMINF_OK;
}

int siminf_launch_info(const siminf_model* m, int32_t out[12]) {
    if (!m || !out) return SIMINF_E_ARG;
    for (int i = 0; i < 12; ++i) out[i] = 0;
    if (m->groups.empty()) return SIMINF_OK;
    const Group& g = m->groups[0];
    out[0] = g.block;
    out[1] = g.blocks;
    out[2] = g.p.lane_queue ? 3 : g.mode;
    out[3] = g.p.pipeline;
    out[4] = m->opt.order;
    out[5] = g.p.nbig;
    out[6] = g.p.pack;
    out[7] = g.p.ngrp;
    out[8] = g.lq_chunk;
    out[9] = (int32_t)g.shmem;
    out[10] = g.lq_chunk ? g.lq_batch : 0;
    out[11] = (int32_t)m->groups.size();
    return SIMINF_OK;
}

int siminf_autotune(siminf_model* m, uint64_t seed, int32_t repeats, void* hip_stream, double* best_ms) {
    if (!m || repeats < 1) return SIMINF_E_ARG;
    if (m->groups.empty()) return SIMINF_OK;
    finish(m);
    struct Cand {
        int block, wide_div, pipeline, pack, grp_div;  // grp_div: see default_group (-1: none)
        int lq;                                        // lane queue: nodes per chunk (0: off)
        int lqb = 16;                                  //             lanes per day-end batch
    };
    auto groups_of = [&](const Group& g, int nb, int gdiv) {
        if (m->opt.group != 0) return m->opt.group < 0 ? g.n : (int)m->opt.group;
        return m->opt.order == 1 ? 0 : default_group(g, nb, gdiv);
    };
    // mean SSA-kernel time of one candidate over `repeats` runs (seeds seed,
    // seed + 1, ...), or a negative value if it cannot be launched: a shape
    // that is fast on most seeds but much slower on some (the heaviest nodes
    // on one lane) is judged by its average
    auto measure = [&](const Cand& c) -> double {
        for (Group& g : m->groups) {
            const int nb = default_wide(m, g, c.wide_div);
            if (configure(m, g, c.block, nb, c.pipeline, m->opt.mode, c.pack, groups_of(g, nb, c.grp_div), c.lq,
                          c.lqb) != SIMINF_OK)
                return -1.0;
        }
        std::vector<double> t;
        for (int r = 0; r < repeats; ++r) {
            double ms[2];
            if (siminf_run(m, seed + (uint64_t)r, 0, hip_stream) != SIMINF_OK || finish(m) != SIMINF_OK ||
                siminf_timing(m, ms) != SIMINF_OK)
                return -1.0;
            t.push_back(ms[0]);
        }
        double sum = 0.0;
        for (double x : t) sum += x;
        return sum / (double)t.size();
    };
    const int pack0 = m->opt.pack ? m->opt.pack : WAVE;
    std::vector<Cand> cands;
    if (m->opt.lane_queue != 1)
        for (int block : {64, 128, 256})
            for (int div : {0, 4, 16, 64})  // wide nodes: none, or work above 1/div of the heaviest
                for (int pipe : {1, 2}) cands.push_back({block, div, pipe, pack0, -1, 0});
    // the lane queue (models without external transfers), at three block
    // sizes and two chunk sizes, unless an option fixes the lane layout
    bool free_only = true;
    for (const Group& g : m->groups)
        free_only = free_only && g.n_e2 == 0 && !g.p.coupled && !is_generated(g.model) && g.p.solver == 0;
    const bool shaped = m->opt.lanes != 0 || m->opt.wide != 0 || m->opt.group != 0 || m->opt.pack != 0;
    if (free_only && m->opt.lane_queue != 2 && (m->opt.lane_queue == 1 || !shaped)) {
        const int ch = m->opt.chunk > 0 ? m->opt.chunk : 512;
        const std::vector<int> batches = m->opt.batch > 0 ? std::vector<int>{m->opt.batch} : std::vector<int>{4, 8, 16};
        for (int block : {64, 128, 256})
            for (int lqb : batches)
                for (int pipe : {2, 1}) cands.push_back({block, 0, pipe, WAVE, -1, ch, lqb});
    }
    if (cands.empty()) return SIMINF_E_UNSUPPORTED;
    double best = 1e300;
    Cand pick = cands[0];
    bool any = false;
    const char* log_env = std::getenv("SIMINF_AUTOTUNE_LOG");
    const bool log = log_env && log_env[0] && log_env[0] != '0';
    auto consider = [&](const Cand& c) {
        const double t = measure(c);
        if (log) {
            std::fprintf(stderr,
                         "siminf_autotune: block %d wide_div %d pipeline %d pack %d group_div %d lane_queue %d/%d: "
                         "%.3f ms\n",
                         c.block, c.wide_div, c.pipeline, c.pack, c.grp_div, c.lq, c.lqb, t);
            std::fflush(stderr);
        }
        if (t >= 0.0 && t < best) {
            best = t;
            pick = c;
            any = true;
        }
    };
    for (const Cand& c : cands) consider(c);
    if (!any) return SIMINF_E_DEVICE;
    // Packing fewer nodes into a wavefront only pays when the device has more
    // SIMDs than a full packing fills: then each wavefront's day ends with the
    // slowest of fewer nodes, and a transfer holds back fewer of them.  Tried
    // on the best shape of the first sweep; the share of wavefront-wide nodes
    // is then tuned again, since cheaper narrow nodes move its optimum.
    long long lanes_needed = 0;
    for (const Group& g : m->groups) lanes_needed += g.n;
    if (pick.lq == 0 && m->opt.pack == 0 && (lanes_needed + WAVE - 1) / WAVE < (long long)device_cus(m) * 4) {
        const Cand first = pick;
        for (int pack : {32, 16, 8, 4}) consider({first.block, first.wide_div, first.pipeline, pack, -1, 0});
        if (pick.pack != first.pack) {
            const Cand second = pick;
            for (int div : {0, 4, 16, 64})
                if (div != second.wide_div) consider({second.block, div, second.pipeline, second.pack, -1, 0});
        }
        // then the heaviest nodes after the wide ones on groups of lanes (the
        // lattice walk on GROUP_LANES lanes): an eighth, a quarter, half or
        // all of them, with the packing chosen so far or 16 or 8 nodes per
        // one-lane wavefront (groups take more wavefronts, and a launch whose
        // wavefronts cannot all be resident drops them)
        if (m->opt.group == 0 && m->opt.order != 1) {
            const Cand third = pick;
            std::vector<int> packs{third.pack};
            if (m->opt.pack == 0)
                for (int pk : {16, 8})
                    if (pk != third.pack) packs.push_back(pk);
            for (int pack : packs)
                for (int gdiv : {8, 4, 2, 1})
                    consider({third.block, third.wide_div, third.pipeline, pack, gdiv, 0});
        }
        // pipelining was chosen on the first sweep's shape: try the other
        // setting on the final one
        Cand last = pick;
        last.pipeline = pick.pipeline == 1 ? 2 : 1;
        consider(last);
    }
    for (Group& g : m->groups) {
        const int nb = default_wide(m, g, pick.wide_div);
        configure(m, g, pick.block, nb, pick.pipeline, m->opt.mode, pick.pack, groups_of(g, nb, pick.grp_div),
                  pick.lq, pick.lqb);
    }
    if (best_ms) *best_ms = best;
    return SIMINF_OK;
}

int siminf_timing(siminf_model* m, double out[2]) {
    if (!m || !out || !m->ran) return SIMINF_E_ARG;
    finish(m);
    float a = 0.f, b = 0.f;
    if (hipEventElapsedTime(&a, m->ev[1], m->ev[2]) != hipSuccess ||
        hipEventElapsedTime(&b, m->ev[0], m->ev[2]) != hipSuccess)
        return SIMINF_E_DEVICE;
    out[0] = a;
    out[1] = b;
    return SIMINF_OK;
}

void siminf_destroy(siminf_model* m) {
    if (!m) return;
    if (m->pending) finish(m);
    for (hipEvent_t e : m->ev)
        if (e) (void)hipEventDestroy(e);
    drop_graph(m);
    for (hipEvent_t e : m->joins)
        if (e) (void)hipEventDestroy(e);
    if (m->fork) (void)hipEventDestroy(m->fork);
    for (hipStream_t ss : m->side)
        if (ss) (void)hipStreamDestroy(ss);
    if (m->h_rp) (void)hipHostFree(m->h_rp);
    if (m->stage) (void)hipFree(m->stage);
    for (void* p : m->owned) (void)hipFree(p);
    delete m;
}

const char* siminf_status_string(int32_t code) {
    switch (code) {
        case SIMINF_OK: return "SIMINF_OK";
        case SIMINF_E_ARG: return "SIMINF_E_ARG";
        case SIMINF_E_UNSUPPORTED: return "SIMINF_E_UNSUPPORTED";
        case SIMINF_E_ALLOC: return "SIMINF_E_ALLOC";
        case SIMINF_E_DEVICE: return "SIMINF_E_DEVICE";
        case SIMINF_E_NEG_STATE: return "SIMINF_E_NEG_STATE";
        case SIMINF_E_BAD_RATE: return "SIMINF_E_BAD_RATE";
        case SIMINF_E_EVENT_OVERDRAW: return "SIMINF_E_EVENT_OVERDRAW";
        case SIMINF_E_EVENT_INDEX: return "SIMINF_E_EVENT_INDEX";
        case SIMINF_E_PTS: return "SIMINF_E_PTS";
        case SIMINF_E_STEP_LIMIT: return "SIMINF_E_STEP_LIMIT";
    }
    return "SIMINF_UNKNOWN";
}

int siminf_prevalence_quantiles(siminf_model* m, int32_t case_c, uint32_t at_risk_mask, int32_t replicates,
                                int32_t k0, int32_t nk, const double* probs, int32_t nq, float* out,
                                void* hip_stream) {
    if (!m || !probs || !out || m->record != SIMINF_RECORD_SUMS || !m->ran) return SIMINF_E_ARG;
    if (replicates < 1 || m->R % replicates != 0 || case_c < 0 || case_c >= m->ncmax || nq < 1 || nk < 0 ||
        k0 < 0 || k0 + nk > m->ntspan || replicates > 4096)
        return SIMINF_E_ARG;
    for (int q = 0; q < nq; ++q)
        if (!(probs[q] >= 0.0 && probs[q] <= 1.0)) return SIMINF_E_ARG;
    double* d_probs = nullptr;
    hipStream_t st = (hipStream_t)hip_stream;
    if (hipMalloc((void**)&d_probs, sizeof(double) * nq) != hipSuccess) return SIMINF_E_ALLOC;
    int rc = SIMINF_OK;
    if (hipMemcpy(d_probs, probs, sizeof(double) * nq, hipMemcpyHostToDevice) != hipSuccess ||
        launch_prevalence(m->d_sums, m->R, m->ntspan, m->ncmax, case_c, at_risk_mask, replicates, k0, nk, d_probs,
                          nq, out, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        rc = SIMINF_E_DEVICE;
    (void)hipFree(d_probs);
    return rc;
}

}  // extern "C"
