// internal.h -- structures shared by the host runtime (runtime.cpp) and the
// kernels (ssa_kernels.hip).  Not part of the public ABI.
#pragma once
#include "device_types.h"

namespace siminf {

constexpr int MAX_NC = 4;     // largest compartment count of the built-in models
constexpr int MAX_NT = 2;     // every built-in model has two transitions
constexpr int WAVE = 64;      // gfx950 wavefront
constexpr int GROUP_LANES = 8;  // lanes of a node carried by a group (8 groups a wavefront)
constexpr int MAX_GROUPS = 8; // one group per built-in model present in a batch

// phases of one unit of time, in the order of Appendix A
enum Phase { PH_SSA = 0, PH_E1 = 1, PH_E2 = 2, PH_PTS = 3 };

// kernel modes
enum Mode { MODE_FREE = 0, MODE_BARRIER = 1, MODE_FLOW = 2 };

// Error key: ordered like the serial algorithm (step, phase, global ordinal),
// code in the low bits.  The global ordinal of a node is its input position
// across runs; of an event, its position in the concatenated event tables.
__host__ __device__ inline uint64_t make_err_key(uint32_t step, uint32_t phase, uint64_t ordinal,
                                                 uint32_t code) {
    return ((uint64_t)step << 44) | ((uint64_t)(phase & 3u) << 42) |
           ((ordinal & ((1ull << 38) - 1)) << 4) | (code & 0xFu);
}
constexpr uint64_t NO_ERROR = ~0ull;
constexpr uint32_t MAX_STEPS = 1u << 20;
constexpr uint64_t MAX_ORDINAL = 1ull << 38;

// Per-run control block in device memory, reset before each run.
struct Ctrl {
    unsigned long long err_key;
    unsigned long long counters[4];  // transitions, node-days, events, SSA draws
    unsigned int work[MAX_GROUPS];   // work-queue cursors (free-running mode)
    unsigned int bar_count;          // grid barrier arrivals
    unsigned int abort;              // set when a wait exceeded its spin limit
    unsigned int e2done;             // dataflow mode: steps whose transfers are applied
    unsigned int pad;
};

// The per-run values a launch reads from device memory rather than from its
// arguments, so that a captured launch sequence serves every run.
struct RunParams {
    unsigned long long seed;
    unsigned int stream_base;
    unsigned int pad;
};

// One scheduled event, packed for a single 16-byte load:
//   x = time, y = type | select mask << 2 | target(c) << (6 + 2c), z = n,
//   w = input index within its spec (the sampling RNG's identity)
// where mask bit c selects compartment c and target(c) is where a sampled
// individual of compartment c goes (c + N[c, shift], or c without shift).
inline int32_t pack_event(int type, uint32_t mask, const int* target, int nc) {
    uint32_t w = (uint32_t)type | (mask << 2);
    for (int c = 0; c < nc; ++c) w |= (uint32_t)target[c] << (6 + 2 * c);
    return (int32_t)w;
}

struct EventSoA {
    const int4* rec;         // packed records
    const double* prop;      // proportion (used when n == 0)
    const int64_t* ordinal;  // global ordinal for the error key
    const int32_t* node;     // barrier mode E2: group-local source node
    const int32_t* dest;     // barrier mode E2: group-local destination
    const int32_t* run;      // E2: run of the event (its sampling stream is stream_base + run)
};

// Position of record m, component c (of width components) of node k in a
// trajectory buffer of ntspan records of n nodes.  The first nmajor nodes,
// each carried by a whole wavefront or a group of lanes, are stored
// node-major so that one node's consecutive records fill the same cache
// lines from one wavefront; the others are stored component-major per
// record, so that the nodes of a wavefront store contiguous runs.
__host__ __device__ inline size_t rec_index(int m, int c, int k, int width, int ntspan, int n, int nmajor) {
    if (k < nmajor) return ((size_t)k * ntspan + m) * width + c;
    return (size_t)nmajor * ntspan * width + ((size_t)m * width + c) * (size_t)(n - nmajor) +
           (size_t)(k - nmajor);
}

// Workgroups are handed to the device's 8 XCDs in turn (workgroup b to XCD
// b mod 8), and each XCD has its own L2.  One-lane-per-node wavefronts store
// a day's record of a compartment as pack consecutive 4-byte words, less
// than a 128-byte cache line when pack < 32; neighbouring wavefronts on
// different XCDs would then write parts of one line from several L2s.  From
// the first whole round of XCDs after the wide nodes' workgroups (a, a
// multiple of 8) on, workgroups are renumbered in spans of 8 g: XCD x takes
// g consecutive ones, which together fill whole lines, while the spans still
// rotate over all XCDs (neighbouring chunks have similar work: the nodes are
// ordered by it).  A bijection: workgroups outside whole spans keep their
// number.
constexpr int XCDS = 8;
__host__ __device__ inline int xcd_block(int b, int b0, int nblk, int g) {
    if (g <= 1) return b;  // (g is 0 when a wavefront's records already fill lines)
    const int a = (b0 + XCDS - 1) / XCDS * XCDS;
    const int span = XCDS * g;
    const int full_end = nblk > a ? a + (nblk - a) / span * span : a;
    if (b < a || b >= full_end) return b;
    const int r = b - a;
    const int rem = r % span;
    return a + (r - rem) + (rem % XCDS) * g + rem / XCDS;
}

// What a node of a spatially coupled model posts for its neighbours each
// day: its continuous state before the post-time step and its size after
// the day's events; `day` (the day step, -1 before the run) is stored last
// with release order and tells a reader the post is complete.  Two posts per
// node (day parity): a node posts day b + 2 only after reading every
// neighbour's day b + 1 post, which each neighbour makes only after reading
// this node's day b post.
struct CplPost {
    double phi;
    int32_t n;
    int32_t day;
};

struct KParams {
    int32_t n;        // nodes in the group
    int32_t nb;       // number of unit-time steps
    int32_t ntspan;
    int32_t mode;     // Mode
    int64_t T1;       // first day boundary
    double t0;        // start time
    uint64_t seed;
    uint32_t stream_base;
    int32_t ngd;
    int32_t S[MAX_NC * MAX_NT];  // state-change matrix, column-major
    uint32_t Gmask[MAX_NT];      // bit k of Gmask[j]: recompute rate k after transition j
    const int32_t* rec_off;      // [nb+1] tspan indices written after step b
    const int32_t* u0;           // [nc][n]
    const double* v0;            // [nv][n]
    int32_t* u;                  // live state [nc][n] (barrier / dataflow modes)
    double* v;                   // [nv][n]
    const double* ld;            // [nld][n]
    const int32_t* node_run;     // [n] run of each node
    const int32_t* node_idx;     // [n] node index within its run
    const int64_t* node_ord;     // [n] global input ordinal
    const double* gdata;         // [nspec][ngd]
    const int32_t* run_spec;     // [runs]
    const int32_t* e1_off;       // [n+1]
    int32_t* e1_cur;             // [n] (barrier mode)
    EventSoA e1;
    const int32_t* e2_step;      // [nb+1] level range of each step
    const int32_t* e2_lvl;       // [levels+1] event range of each level
    EventSoA e2;
    const int32_t* e2n_off;      // dataflow: [n+1] per node, its external transfers
    const int4* e2n_rec;         //           packed record of each (sources sample from it)
    const int4* e2n_item;        //           x = event index, y = step, z = role (0 source,
                                 //           1 destination, 2 both), w = run of the event
    unsigned long long* mail;    // dataflow: [n_e2] counts a transfer delivers (0 = not yet)
    int32_t* mail_big;           //           [n_e2][Nc] counts too large to pack
    int32_t n_e2;
    int32_t record;              // 0 full, 1 sums
    int32_t sums_nc;             // compartment stride of the sums array
    int32_t* U;                  // [ntspan][nc][n]
    double* V;                   // [ntspan][nv][n]
    unsigned long long* sums;    // [runs][ntspan][sums_nc]
    Ctrl* ctrl;
    int32_t group;
    int32_t nchunks;             // chunks of the free-running work queue
    int32_t pack;                // nodes per wavefront that carries one lane per node
                                 // (64, 32, 16, 8 or 4; the other lanes idle)
    int32_t nblocks;
    int32_t pipeline;            // 1: overlap the next step's random numbers with this step
    int32_t nbig;                // the first nbig nodes each get a whole wavefront
    int32_t ngrp;                // the next ngrp nodes get a group of lanes each (the
    int32_t ngw;                 //   lattice walk on a group), ngw wavefronts of them
    int32_t nmajor;              // nbig + ngrp: nodes whose records are node-major
    int32_t lattice;             // wide nodes walk a lattice of reachable states
    uint64_t wait_ticks;         // wall-clock ticks one wait may last before abort
    const RunParams* rp;         // seed and stream base of the current run (device)
    int32_t lane_queue;          // free-running, one lane per node, each lane advancing its
                                 // own node and taking the next node of its chunk when done
    int32_t nlchunks;            // lane-queue chunks (runs cut into pieces of consecutive nodes)
    const int4* lchunks;         // [nlchunks] x = first node, y = end, z = run
    int32_t lq_batch;            // lanes that wait at their day's end before the
                                 // wavefront closes their days together
    int32_t solver;              // 0 the direct method, 1 the all events method:
    int32_t nt;                  //   transitions, and per node and channel
    double* aem_T;               //   [nt][n] the integrated rate,
    double* aem_P;               //   [nt][n] the level of the next firing,
    uint32_t* aem_K;             //   [nt][n] the index of the next exponential
    int32_t coupled;             // spatial coupling of the post-time step (SISe_sp):
    const int32_t* cpl_off;      //   [n+1] each node's neighbours (internal order), then
                                 //         the nodes that list it but that it does not list
    const int32_t* cpl_fend;     //   [n]   end of the first part (the summed neighbours)
    const int32_t* cpl_idx;      //   [nnz] neighbour
    const double* cpl_w;         //   [nnz] coupling weight D / distance
    CplPost* cpl_post;           //   [2][n] the day's posts
};

// Lane-queue kernel: recording slots per wavefront (a slot accumulates one
// chunk's per-run sums in LDS) and the LDS budget of a workgroup for them.
constexpr int LQ_SLOTS = 2;
constexpr int LQ_LDS_BYTES = 64 * 1024;

// Launchers implemented in ssa_kernels.hip.
#ifndef __HIPCC_RTC__
hipError_t launch_init(const KParams& p, int nc, int nv, int first_rec, bool reset_ctrl,
                       const unsigned long long* sums_init, long long sums_len, hipStream_t st);
hipError_t launch_group(int model, const KParams& p, int block, int blocks, size_t shmem,
                        hipStream_t st);
int max_blocks_per_cu(int model, int mode, int pipeline, bool grp, int block, size_t shmem,
                      bool lane_queue = false, bool aem = false);
hipError_t launch_gather(int nc, int nv, const int32_t* U, const double* V, int n, int ntspan, int nmajor,
                         const int32_t* pos, int nn, int32_t* Uo, double* Vo, hipStream_t st);
hipError_t launch_sparse_gather(const int32_t* U, const double* V, int width, int n, int ntspan, int nmajor,
                                const int32_t* pos, const int64_t* col_ptr, const int32_t* row_idx, long long nnz,
                                double* out, hipStream_t st);
// generated models (generated.cpp): launch through the run-time compiled module
hipError_t generated_launch(int id, const KParams& p, int block, int blocks, size_t shmem, hipStream_t st);
int generated_blocks_per_cu(int id, int mode, int pipeline, int block, size_t shmem, bool aem);
hipError_t launch_prevalence(const unsigned long long* sums, int runs, int ntspan, int nc,
                             int case_c, uint32_t mask, int reps, int k0, int nk,
                             const double* probs, int nq, float* out, hipStream_t st);
#endif  // __HIPCC_RTC__

}  // namespace siminf
