/*
 * siminf.h -- C ABI of libsiminf.so, an MI355X (gfx950) implementation of
 * the split-step stochastic simulation of Widgren, Bauer, Eriksson &
 * Engblom, "SimInf: An R package for data-driven stochastic disease spread
 * simulations" (arXiv 1605.01421).
 *
 * What a run computes (section 2.3, eqs. numstep1-numstep3; Appendix A):
 * every node (sub-population) i holds an integer compartment vector u[,i]
 * (and optionally a real vector v[,i]).  Time advances one unit ("day") at a
 * time.  Within a day each node runs Gillespie's direct method: sum of the
 * transition rates lambda, waiting time tau = -log(r1)/lambda, stop when the
 * next transition would pass the day boundary, otherwise pick transition n
 * by inversion with r2, add column S[,n] to u[,i] and recompute the rates
 * that the dependency graph G marks.  At the boundary the node's scheduled
 * exit / enter / internal-transfer events (E1) are applied, then -- after
 * all nodes reached the boundary -- the external transfers (E2) in table
 * order, then the post-time-step function updates v[,i] (section 3.4).
 * U and V are recorded whenever time passes a tspan point (Table 1).
 *
 * Random numbers are Philox4x32-10 blocks (Salmon et al., SC'11) used as a
 * keyed counter function: key = seed; SSA step k of node i (0-based within
 * its run) while advancing towards integer day T uses counter
 * (k, (uint32)T, i, stream & 0xFFFFFF); event sampling of the event with
 * input index e uses counters (b, 0, e, (stream & 0xFFFFFF) | 1<<24) for
 * blocks b = 0, 1, ...  Results therefore do not depend on the launch shape.
 * Uniforms: r = (k + 1/2) 2^-52 with k = (w_a << 20) | (w_b >> 12); r1 from
 * words 0,1 and r2 from words 2,3 of the step's block.  log(r1) is the
 * library's own series logarithm (reduction of the argument to
 * [sqrt(1/2), sqrt(2)] times a power of two, the atanh series up to s^23,
 * ln 2 in two parts), every operation one IEEE binary64 rounding.  Sampling
 * without replacement draws one individual at a time with Lemire's unbiased
 * bounded integer on successive 32-bit words.
 *
 * Conventions: every function returns an int status, 0 on success and one
 * of the negative SIMINF_E_* codes otherwise; none aborts the process.
 * Indices are 0-based; shift = -1 means "no shift".  Matrices are dense and
 * column-major as in the paper (S is Nc x Nt, element (c, j) at S[c + j*Nc];
 * u0 is Nc x Nn, node i's compartments at u0[c + i*Nc]).  A handle is used
 * by one host thread at a time; separate handles are independent.
 */
#ifndef SIMINF_H
#define SIMINF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ----------------------------------------------------- */
enum {
    SIMINF_OK = 0,
    SIMINF_E_ARG = -1,            /* invalid argument or model (validity check, section 3.4.2) */
    SIMINF_E_UNSUPPORTED = -2,    /* model id or size outside what the library implements */
    SIMINF_E_ALLOC = -3,          /* device or host allocation failed */
    SIMINF_E_DEVICE = -4,         /* HIP runtime error, or an in-kernel barrier timed out */
    SIMINF_E_NEG_STATE = -5,      /* a transition made a compartment negative (App. A, 17) */
    SIMINF_E_BAD_RATE = -6,       /* a transition rate was negative or not finite (App. A: the
                                     rates must be valid propensities) */
    SIMINF_E_EVENT_OVERDRAW = -7, /* an event asked for more individuals than exist (sec. 4.1.2) */
    SIMINF_E_EVENT_INDEX = -8,    /* an event names a node / select / shift out of range */
    SIMINF_E_PTS = -9,            /* the post-time-step function failed (non-finite state) */
    SIMINF_E_STEP_LIMIT = -10     /* implementation limit, not the method's: a node needed more
                                     than 2^24 SSA draws within one unit of time (the draw index
                                     is the first Philox counter word; see siminf_run) */
};

/* ---- built-in models (the TRFun / PTSFun pairs of section 3.4.1) ----------
 * SIR (eq. SIR): Nc=3 (S,I,R), Nt=2, gdata=(beta, gamma), Nv=0, Nld=0.
 *    S->I at beta*S*I/(S+I+R) (0 when the node is empty), I->R at gamma*I.
 * SIS (eqs. sirtrans, SIRstoich): Nc=2, Nt=2, gdata=(beta, gamma).
 *    S+I->2I at beta*S*I, I->S at gamma*I.
 * SISE (sec. 4.2 without spatial coupling): Nc=2, Nt=2, Nv=1 (phi),
 *    Nld=4 (day of year each season ends), gdata=(upsilon, gamma, alpha,
 *    beta_1..beta_4).  S->I at upsilon*phi*S, I->S at gamma*I; after each day
 *    phi <- phi*(1-beta_q) + alpha*I/(S+I) (0 for an empty node), q = first
 *    season whose end is >= the day of year of the new day (else season 1).
 * SISE_SP (sec. 4.2, eq. envInfPressure-local-spread): SISE with the spatial
 *    coupling of phi among proximal nodes; gdata = (upsilon, gamma, alpha,
 *    beta_1..beta_4, D), the sparse distance matrix in the spec's nb_*
 *    fields.  After each day
 *      phi_i <- (phi_i*(1-beta_q) + alpha*I_i/N_i) + c_i,
 *      c_i = sum over i's neighbours k, in stored order, of
 *            ((phi_k*N_k - phi_i*N_i) / N_i) * (D / d_ik),
 *    all phi taken before the day's update, N = S+I after the day's events
 *    (the alpha term and c_i are 0 for an empty node).  The nodes then
 *    depend on each other every day: such a model runs only in the dataflow
 *    kernel (all its node wavefronts resident on the device at once, else
 *    SIMINF_E_UNSUPPORTED) and alone in its handle (no other model group).
 * BIRTH_DEATH: Nc=1, Nt=2, gdata=(b, d): X->2X at b*X, X->0 at d*X.
 * IMMIGRATION_DEATH: Nc=1, Nt=2, gdata=(kappa, mu): 0->X at kappa, X->0 at mu*X.
 * Arithmetic is IEEE binary64 in the operation order written above. */
enum {
    SIMINF_SIR = 0,
    SIMINF_SIS = 1,
    SIMINF_SISE = 2,
    SIMINF_BIRTH_DEATH = 3,
    SIMINF_IMMIGRATION_DEATH = 4,
    SIMINF_SISE_SP = 5
};

/* ---- generated models (section 5.1, the model parser) ----------------------
 * A model given as transition strings "from -> propensity -> to" over named
 * compartments, global data (gdata), local data (ldata) and continuous state
 * (v).  `from` and `to` are "@" (the empty set) or terms "X" or "k*X"
 * (k >= 1) joined by '+'; column j of S is to - from.  The propensity is an
 * expression in numbers, those names, + - * / (left-associative, * and /
 * before + and -), unary - and +, and parentheses, evaluated in IEEE
 * binary64 in the order of its parse tree with every name read as binary64
 * (compartment counts converted exactly).  G[k][j] (rate k recomputed after
 * transition j, stored column-major as G[k + j*Nt]) is set when propensity k
 * reads a compartment that transition j changes.  E and N (select and shift
 * matrices of the scheduled events, Table 2) are part of the definition:
 * they are compiled into the model.  The post-time step of a generated model
 * leaves v unchanged.
 * siminf_define_model parses the definition, writes S (Nc x Nt) and G
 * (Nt x Nt) when the pointers are not NULL, and compiles the kernels for it
 * at run time (hipRTC, gfx950; a few seconds); *model_id is then the value
 * for siminf_spec.model (the spec's S and G must equal the ones written here,
 * and a spec with events must carry this E and N).  Returns SIMINF_E_ARG with
 * the reason in msg (may be NULL) for a definition that does not parse,
 * SIMINF_E_DEVICE with the compiler's log for a failed compilation, and
 * SIMINF_E_UNSUPPORTED once SIMINF_GEN_LAST - SIMINF_GEN_FIRST + 1 models
 * exist in the process.  Definitions are kept until the process ends; a
 * generated model runs one lane per node (the free-running, barrier and
 * dataflow kernels; not the lane queue, wavefront-wide nodes or groups). */
enum {
    SIMINF_GEN_FIRST = 64,
    SIMINF_GEN_LAST = 127,
    SIMINF_GEN_MAX_NC = 16,
    SIMINF_GEN_MAX_NT = 32
};
typedef struct {
    int32_t nt;                        /* transitions, "from -> propensity -> to" */
    const char *const *transitions;
    int32_t nc;                        /* compartment names (the rows of S, E, N) */
    const char *const *compartments;
    int32_t ngd;                       /* names of gdata[0..ngd) */
    const char *const *gdata_names;
    int32_t nld;                       /* names of ldata[0..nld) of a node */
    const char *const *ldata_names;
    int32_t nv;                        /* names of v[0..nv) of a node */
    const char *const *v_names;
    int32_t Ecols;                     /* select matrix, nc x Ecols column-major (0/1) */
    const int32_t *E;
    int32_t Ncols;                     /* shift matrix, nc x Ncols column-major */
    const int32_t *N;
} siminf_model_def;
int siminf_define_model(const siminf_model_def *def, int32_t *model_id, int32_t *S_out, int32_t *G_out,
                        char *msg, size_t msg_cap);
/* The generated source of a model (the model type the kernels were compiled
 * for); *needed is its length plus one. */
int siminf_generated_source(int32_t model_id, char *buf, size_t cap, size_t *needed);

/* event type codes (Table 2) */
enum { SIMINF_EXIT = 0, SIMINF_ENTER = 1, SIMINF_INTTRANS = 2, SIMINF_EXTTRANS = 3 };

/* what a run records at each tspan point */
enum {
    SIMINF_RECORD_FULL = 0, /* U (and V) for every node: siminf_trajectory */
    SIMINF_RECORD_SUMS = 1  /* per run, the sum over nodes of each compartment: siminf_sums */
};

/* One model run's inputs (Tables 1 and 2).  All pointers are host memory
 * owned by the caller; siminf_create copies them and keeps no reference.
 *   S      Nc x Nt  state-change matrix (column j added when transition j fires)
 *   G      Nt x Nt  dependency graph: G[k + j*Nt] != 0 means rate k is
 *                   recomputed after transition j
 *   u0     Nc x Nn  initial compartments (>= 0)
 *   v0     Nv x Nn  initial continuous state
 *   ldata  Nld x Nn local data;  gdata  Ngd global data
 *   tspan  Ntspan strictly increasing output times; tspan[0] is the start,
 *          tspan[Ntspan-1] the end.  Time advances in unit steps to the
 *          integer days floor(tspan[0])+1, ..., ceil(tspan[Ntspan-1]).
 *   events Nev rows: ev_type (SIMINF_EXIT..EXTTRANS), ev_time (integer day;
 *          an event is applied at the first day boundary T >= ev_time, so
 *          events at or before tspan[0] are applied at the first boundary),
 *          ev_node, ev_dest (external transfers only), ev_n (>= 0; 0 means
 *          round(ev_prop * selected total), half away from zero), ev_prop in
 *          [0, 1], ev_select (column of E), ev_shift (column of N, or -1).
 *   E      Nc x Ecols select matrix; N  Nc x Ncols shift matrix (Table 2).
 * Same-day order: exit < enter < internal transfer (per node, in the
 * node's own lane) < external transfer (all nodes, in input order). */
typedef struct {
    int32_t model, Nc, Nt, Nn, Nv, Nld, Ngd, Ntspan;
    const int32_t *S, *G, *u0;
    const double *v0, *ldata, *gdata, *tspan;
    int32_t Nev, Ecols, Ncols;
    const int32_t *ev_type, *ev_time, *ev_node, *ev_dest, *ev_n, *ev_select, *ev_shift;
    const double *ev_prop;
    const int32_t *E, *N;
    /* SISE_SP only (ignored otherwise): the distance matrix of section 4.2
     * (distance_matrix() with its cutoff) in compressed columns -- node i's
     * neighbours are nb_idx[nb_ptr[i] .. nb_ptr[i+1]-1] (0-based, the same
     * run) at distances nb_dist > 0 in the same positions; nb_ptr has Nn+1
     * entries, nb_ptr[0] = 0, nb_ptr[Nn] = Nnb. */
    int32_t Nnb;
    const int32_t *nb_ptr, *nb_idx;
    const double *nb_dist;
} siminf_spec;

/* Launch and recording options; a zeroed struct (or NULL) gives defaults. */
typedef struct {
    int32_t record;    /* SIMINF_RECORD_FULL (default) or SIMINF_RECORD_SUMS */
    int32_t block;     /* threads per workgroup: 64, 128, 192 or 256; 0 = chosen
                          from the model (64 with external transfers, else 256) */
    int32_t order;     /* lane order: 0 = binned by expected work (default), 1 = input order */
    int32_t lanes;     /* lanes per node: 0 auto, 1 one lane for every node, 64 the
                          heaviest nodes get a whole wavefront (its 64 lanes draw
                          64 steps' random numbers at once) */
    int32_t max_blocks;/* cap on the number of workgroups (0 = occupancy limit) */
    int32_t pipeline;  /* 0 auto, 1 overlap each step's random numbers with the
                          previous step (latency), 2 off (throughput) */
    int32_t mode;      /* runs with external transfers: 0 auto, 1 grid-barrier
                          kernel, 2 dataflow kernel (node state in registers) */
    int32_t wide;      /* with lanes = 64: how many of the heaviest nodes get a
                          wavefront (0 = chosen from the expected work) */
    int32_t lattice;   /* wavefront-wide nodes: 0 auto (on when G marks both rates
                          after either transition), 1 the same, 2 off (every
                          step on one dependent chain); the results are equal */
    int32_t wait_ms;   /* longest wall-clock time one wait inside a kernel (a
                          grid barrier, or a destination waiting for its source's
                          transfer) may take before the run is abandoned with
                          SIMINF_E_DEVICE; 0 = 60000.  Legitimate waits can last
                          as long as the slowest node's share of the run. */
    int32_t graph;     /* 1: the first siminf_run captures the run's launches in a
                          HIP graph and every run replays it (the seed and stream
                          base are read from device memory); only for models
                          without external transfers, else siminf_run returns
                          SIMINF_E_UNSUPPORTED.  Reconfiguring (siminf_autotune)
                          drops the graph.  siminf_timing's kernel time then also
                          covers the short init kernel.  0 (default): plain
                          launches. */
    int32_t pack;      /* nodes in a wavefront that gives each node one lane: 64,
                          32, 16, 8 or 4 (the remaining lanes idle); 0 auto: 64,
                          unless the device has more CUs than wavefronts, then
                          the largest packing that gives each SIMD a wavefront
                          (at least 16 with SISe_sp coupling; 4 if none does),
                          raised again where the dataflow kernel cannot hold
                          every wavefront.  Fewer
                          nodes per wavefront shorten a latency-bound run (each
                          wavefront's day ends with its slowest node, and an
                          external transfer holds back only the destination's
                          wavefront) when the device has SIMDs to spare.  The
                          grid-barrier kernel always packs 64; the results do
                          not depend on it. */
    int32_t group;     /* how many nodes after the wavefront-wide ones get a
                          group of 8 lanes each (8 nodes a wavefront), on
                          which the lattice walk covers 3 steps per pass: 0
                          none (the autotuner may choose some), -1 all, else
                          that many.  Only where the lattice walk applies (see
                          lattice) and not in the grid-barrier kernel; the
                          results do not depend on it. */
    int32_t lane_queue;/* models without external transfers: 1 every node on one
                          lane that advances its node day by day on its own and,
                          when the node is done, takes the next node of its
                          wavefront's chunk (the throughput kernel); 2 off (the
                          lanes of a wavefront go through each day together);
                          0 auto: on when no lanes, wide, group or pack option
                          is set and the model has at least 64 nodes per SIMD
                          of the device.  With SIMINF_RECORD_SUMS it needs
                          2 x Ntspan x Nc x 8 bytes of LDS per wavefront (at
                          most 64 KiB per workgroup), else SIMINF_E_UNSUPPORTED
                          (auto: off).  The results do not depend on it. */
    int32_t chunk;     /* lane queue: nodes per chunk (consecutive nodes of one
                          run handed to one wavefront), 64..1048576; 0 = 512 */
    int32_t batch;     /* lane queue: lanes of a wavefront that wait at the end
                          of a day (or without a node) before the wavefront
                          serves them together, 1..64; 0 = 16 */
    int32_t solver;    /* section 3.4: 0 the split-step direct method (default);
                          1 the all events method: every transition channel
                          of a node fires when its integrated rate reaches
                          the running sum of unit exponentials drawn from the
                          channel's own stream (Philox block (k, j, node,
                          stream | 2<<24), -log of the uniform from its first
                          two words, k = 0, 1, ... per channel); the channel
                          with the least (P_j - T_j)/w_j fires, the lowest j
                          on a tie, unless that time crosses the day
                          boundary, where every integral advances to it and
                          carries over.  Same law, other draws; one lane per
                          node (no lane queue, wavefront-wide nodes or
                          groups); checks and error keys as the direct
                          method's.  Anything else: SIMINF_E_ARG. */
} siminf_options;

typedef struct siminf_model siminf_model;

/* Validates one run (the validity check of section 3.4.2), copies it to
 * device memory of the current HIP device and returns a handle in *out.
 * Static event errors are reported here: SIMINF_E_EVENT_INDEX for a node,
 * dest, select or shift out of range (also a shift target outside 0..Nc-1
 * for any selected compartment); siminf_error_info then names the event.
 * Shape: Nc, Nt and Nv must equal the built-in model's (SIR 3/2/0, SIS 2/2/0,
 * SISe 2/2/1, birth-death and immigration-death 1/2/0; anything else is
 * SIMINF_E_ARG), Nld and Ngd at least the model's; Ntspan >= 1, Nn >= 0. */
int siminf_create(const siminf_spec *spec, const siminf_options *opt, siminf_model **out);

/* A batch: specs[s] is run replicates[s] times (run r of the batch uses
 * stream_base + r in siminf_run; runs are numbered spec by spec).  All specs
 * share tspan; specs of the same model must share S, G, E and N.  External
 * transfers are allowed only when every spec is the same model.  Each run's
 * results equal a single-run siminf_create/siminf_run of that spec with
 * stream = stream_base + r. */
int siminf_create_batch(const siminf_spec *specs, int32_t nspecs, const int32_t *replicates,
                        const siminf_options *opt, siminf_model **out);

/* Enqueues one complete run on hip_stream (a hipStream_t; NULL = the null
 * stream) and returns without waiting: the whole of run() in section 3.4.2
 * and the Appendix A algorithm -- for every unit of time from
 * floor(tspan[0]) + 1 to ceil(tspan[Ntspan-1]), the direct-method SSA of
 * every node up to the boundary, the node's exit / enter / internal-transfer
 * events, the external transfers in table order, the post-time-step
 * function, and the U/V records of the tspan points passed (section 3.3,
 * eq. numstep3, Table 1).  seed is the Philox key (the paper's GSL seed);
 * run r of the handle uses stream stream_base + r, and stream_base + runs
 * must not exceed 2^24.  Draws are keyed by the absolute day (the counter
 * word (uint32)T), so a simulation split into consecutive runs that each
 * start from the previous one's last state equals one run over the whole
 * span: this replaces a day-offset argument.  Runs of the same handle must
 * not overlap; a new run first waits for the previous one.  Errors in the
 * run are reported by siminf_wait; this call returns SIMINF_E_ARG for a bad
 * stream range, SIMINF_E_UNSUPPORTED when options.graph is set for a model
 * with external transfers, SIMINF_E_DEVICE when a launch fails.  Each node-
 * day may take at most 2^24 SSA draws (SIMINF_E_STEP_LIMIT). */
int siminf_run(siminf_model *m, uint64_t seed, uint32_t stream_base, void *hip_stream);

/* Waits for the last run and returns its status: 0 or the code of the first
 * error in the serial order of Appendix A (day step, then phase SSA < E1 < E2
 * < PTS, then node or event index), which siminf_error_info describes; a
 * failing run stops after that day.  SIMINF_E_DEVICE if a kernel failed or a
 * wait inside it passed options.wait_ms. */
int siminf_wait(siminf_model *m);

/* The trajectory of section 3.4.2 (trajectory(), Table 1): copies run
 * `run`'s recorded U (Nc*Nn x Ntspan, column-major: node i's compartment c at
 * tspan[k] is U[c + i*Nc + k*Nc*Nn]) and V (Nv*Nn x Ntspan, same layout) to
 * U / V (either may be NULL).  dst_is_device != 0 means U and V are device
 * pointers on the model's device; otherwise host memory owned by the caller
 * (staged through a device buffer the handle keeps for later calls).  Waits
 * for the last run (synchronising only its stream).  Requires
 * SIMINF_RECORD_FULL, else SIMINF_E_ARG.  Returns the run's status: after a
 * failed run the records are copied too, but those after the failing day are
 * undefined. */
int siminf_trajectory(siminf_model *m, int32_t run, int32_t *U, double *V, int32_t dst_is_device);

/* Selected entries of run `run`'s trajectory (Table 1, U_sparse and
 * V_sparse): the nonzero pattern of a sparse (Nn*width) x Ntspan matrix in
 * compressed columns -- col_ptr[0..Ntspan] (col_ptr[0] = 0, nondecreasing,
 * col_ptr[Ntspan] = nnz) and row_idx[0..nnz), row = node*width + c in the
 * run's own node numbering -- and the values written, as binary64, to
 * values[0..nnz) in pattern order: U (which = 0, width Nc) or V (which = 1,
 * width Nv) at tspan index m for the entries of column m.  The pattern is
 * host memory; values is host memory, or device memory when dst_is_device.
 * The model records in SIMINF_RECORD_FULL (the full trajectory stays on the
 * device; only the selected entries are copied out).  Returns SIMINF_E_ARG
 * for a bad pattern (checked before any device work), else as
 * siminf_trajectory. */
int siminf_trajectory_sparse(siminf_model *m, int32_t run, int32_t which, int64_t nnz, const int64_t *col_ptr,
                             const int32_t *row_idx, double *values, int32_t dst_is_device);

/* Copies the per-run compartment sums over all nodes at each tspan point
 * (the numerators and denominators of prevalence() in section 4.2), int64
 * [runs][Ntspan][Nc] row-major, to sums (host, or device if dst_is_device).
 * Requires SIMINF_RECORD_SUMS, else SIMINF_E_ARG.  Returns the run's status
 * like siminf_trajectory. */
int siminf_sums(siminf_model *m, int64_t *sums, int32_t dst_is_device);

/* Counters of the last run (Appendix A): out[0] transitions executed
 * (line 17 of each step that stays inside the day), out[1] node-days
 * simulated, out[2] scheduled events applied (section 3.3), out[3] SSA
 * draws (Philox blocks: the transitions plus each node-day's final draw
 * whose step crosses the boundary).  Waits for the last run; after a failed
 * run they count the work done up to the failure in each node. */
int siminf_counters(siminf_model *m, uint64_t out[4]);

/* Sizes of a handle: out[0] runs, out[1] total nodes, out[2] Ntspan,
 * out[3] Nc (largest over specs), out[4] Nv (largest), out[5] day steps. */
int siminf_shape(const siminf_model *m, int64_t out[6]);

/* First error of the last run (or of create), in the serial order of
 * Appendix A and the error rules of sections 3.3 and 3.4: code, 0-based day
 * step, phase (0 SSA, 1 E1, 2 E2, 3 PTS; -1 = create), index (node within
 * its run for SSA/PTS, event input index for events and for a static event
 * error found by create) and run.  Any pointer may be NULL. */
int siminf_error_info(const siminf_model *m, int32_t *code, int64_t *step, int32_t *phase,
                      int64_t *index, int32_t *run);

/* The same error as a NUL-terminated message of at most cap bytes (cap > 0)
 * in buf, owned by the caller, e.g. "SIMINF_E_EVENT_OVERDRAW at day step 37
 * in an external transfer, event 1234 of run 0: an event asked for more
 * individuals than the selected compartments hold"; "SIMINF_OK" when there
 * was none.  A longer message is truncated. */
int siminf_error_message(const siminf_model *m, char *buf, size_t cap);

/* Launch configuration chosen for the handle (its first model group):
 * out[0] threads per block, out[1] blocks, out[2] kernel (0 free-running,
 * 1 grid-barrier, 2 dataflow, 3 lane queue), out[3] pipelining on/off,
 * out[4] order, out[5] nodes carried by a whole wavefront, out[6] nodes per
 * wavefront of the one-lane-per-node ones (the pack option), out[7] nodes
 * on a group of lanes (the group option), out[8] lane queue: nodes per
 * chunk (0 = not the lane queue), out[9] dynamic LDS bytes per workgroup,
 * out[10] lane queue: the batch option in use, out[11] model groups. */
int siminf_launch_info(const siminf_model *m, int32_t out[12]);

/* Autotuner: runs the model `repeats` times for each candidate launch shape
 * (threads per block 64/128/256; no wavefront-wide nodes, or those whose
 * expected work exceeds 1/4, 1/16 or 1/64 of the heaviest node's;
 * pipelining on/off), on hip_stream with seeds seed, seed+1, ..., and keeps
 * the shape with the smallest mean SSA-kernel time over the repeats
 * (written to *best_ms if not NULL).  With pack = 0 and fewer
 * nodes than the device has SIMDs times 64, it then tries 32, 16, 8 and 4
 * nodes per wavefront on the best shape and, if one of those wins, the four
 * wide-node choices again with it; then (with group = 0) groups of lanes for
 * the heaviest eighth, quarter or half of the nodes after the wide ones, or
 * for all of them, each with the packing chosen so far and with 16 and 8
 * nodes per one-lane wavefront, and finally the other pipelining setting on
 * the best shape.  Every shape gives bit-identical results;
 * the handle's recorded results are overwritten.  With the environment
 * variable SIMINF_AUTOTUNE_LOG set (and not "0"), each candidate's time is
 * printed to stderr as it is measured. */
int siminf_autotune(siminf_model *m, uint64_t seed, int32_t repeats, void *hip_stream, double *best_ms);

/* Device time of the last run, from HIP events the library records on the
 * run's stream: out[0] milliseconds of the SSA kernels (all days, events,
 * post-time steps and records), out[1] of the whole run including the
 * per-run initialisation.  Waits for the last run. */
int siminf_timing(siminf_model *m, double out[2]);

/* Frees the handle and its device memory (waits for its last run).  Call it
 * while the HIP runtime is alive (before the process starts to exit); a
 * handle left open at exit is reclaimed with the process. */
void siminf_destroy(siminf_model *m);

/* Status code name, e.g. "SIMINF_E_EVENT_OVERDRAW". */
const char *siminf_status_string(int32_t code);

/* ---- prevalence and quantiles (section 4.2, prevalence(); surrogate targets)
 * For a SIMINF_RECORD_SUMS batch whose runs are grouped in sets of
 * `replicates` consecutive runs: population prevalence
 *     P[r][k] = sums[r][k][case_c] / sum_{c in at_risk} sums[r][k][c]
 * (0 when the denominator is 0) for the tspan indices k = k0, k0+1, ...,
 * k0+nk-1, then for every set and k the type-7 quantiles (linear
 * interpolation between order statistics, h = (R-1) p) at the nq
 * probabilities `probs`, written as float out[set][k-k0][q] (device
 * pointer).  at_risk_mask has bit c set for each compartment in the
 * denominator.  Computed in binary64 and rounded once to float. */
int siminf_prevalence_quantiles(siminf_model *m, int32_t case_c, uint32_t at_risk_mask,
                                int32_t replicates, int32_t k0, int32_t nk,
                                const double *probs, int32_t nq, float *out, void *hip_stream);

/* ---- surrogate network (BF16 matrix cores, FP32 accumulation) -------------
 * A multilayer perceptron dims[0] -> dims[1] -> ... -> dims[nlayers]:
 *   Z_l = A_{l-1} W_l^T + b_l,  A_l = GELU(Z_l) (exact erf form) for hidden
 *   layers, output Y = Z_L.  Products take bfloat16 operands (inputs,
 *   weights, activations, gradients, rounded to nearest even) and accumulate
 *   in float32; master weights and optimiser state are float32.
 * Training minimises the pinball (quantile) loss averaged over batch and
 * outputs, mean max(q_j (t - y), (q_j - 1)(t - y)) with q_j = probs[j mod nq],
 * using AdamW.  The network owns its device memory; X, T and Y are device
 * pointers (float32, row-major [batch][features]).  Not thread-safe per handle. */
typedef struct siminf_mlp siminf_mlp;

/* Creates a network with zero weights for batches up to max_batch. */
int siminf_mlp_create(int32_t nlayers, const int32_t *dims, int32_t max_batch, siminf_mlp **out);

/* Sets layer `layer`'s weights W (dims[l+1] x dims[l], row-major, host
 * float32) and bias b (host), refreshes the bfloat16 copy and resets the
 * layer's optimiser state and the step count. */
int siminf_mlp_set_params(siminf_mlp *m, int32_t layer, const float *W, const float *b);

/* Copies the float32 master weights and bias of a layer to host memory. */
int siminf_mlp_get_params(const siminf_mlp *m, int32_t layer, float *W, float *b);

/* Y[B][dims[L]] = network(X[B][dims[0]]), enqueued on hip_stream. */
int siminf_mlp_forward(siminf_mlp *m, const float *X, int32_t B, float *Y, void *hip_stream);

/* Forward, pinball loss against targets T[B][dims[L]] at quantile levels
 * probs[0..nq-1] (nq <= 8), and back-propagation; the gradients stay in the
 * handle (siminf_mlp_get_grads, siminf_mlp_adamw).  If loss is not NULL the
 * call waits and stores the mean loss there. */
int siminf_mlp_backward(siminf_mlp *m, const float *X, const float *T, int32_t B, const double *probs,
                        int32_t nq, double *loss, void *hip_stream);

/* Copies the last computed gradients of a layer to host memory (waits). */
int siminf_mlp_get_grads(const siminf_mlp *m, int32_t layer, float *dW, float *db);

/* One AdamW step (decoupled weight decay) of every layer with the last
 * gradients: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * w -= lr (m/(1-b1^t) / (sqrt(v/(1-b2^t)) + eps) + weight_decay w). */
int siminf_mlp_adamw(siminf_mlp *m, float lr, float beta1, float beta2, float eps, float weight_decay,
                     void *hip_stream);

/* Frees the network (waits for the device). */
void siminf_mlp_destroy(siminf_mlp *m);

/* The surrogate's answer from an ensemble of `members` networks of the same
 * input and output widths (the learned part of the build, not in the
 * paper): each member maps X[B][dims[0]] (device, float32, standardised
 * inputs) to standardised outputs p; per output j, y = p * y_std[j] +
 * y_mean[j] (device float32 vectors of the output width), then
 *   Y[b][j]          = mean of y over the members (device float32 [B][N]),
 *   disagreement[b]  = mean over j of the members' sample standard deviation
 *                      of y (divisor members - 1; 0 for one member),
 * computed in binary64 and rounded once to float32.  Enqueued on hip_stream;
 * a device workspace of members x B x N floats is taken from the stream's
 * memory pool for the call.  1 <= members <= 64, B >= 1 (any size: members
 * run in slices of their largest batch); SIMINF_E_ARG for mismatched widths
 * or null pointers.  Uses each member's activation buffers: no other work
 * on those networks may overlap the call. */
int siminf_mlp_ensemble_predict(siminf_mlp *const *nets, int32_t members, const float *X, int32_t B,
                                const float *y_mean, const float *y_std, float *Y, float *disagreement,
                                void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation as siminf_mlp_ensemble_predict, with the members x B x N
 * workspace in a fixed array of 2^22 floats (16 MiB) in device memory that
 * the library keeps on each device until the process ends; no allocation of
 * any kind.  members x B x N above 2^22 returns SIMINF_E_UNSUPPORTED before
 * any work is enqueued.  Every call on one device shares that array:
 * calls that overlap on one device (other streams or threads) race and must
 * be serialised by the caller. */
int siminf_mlp_ensemble_predict_static(siminf_mlp *const *nets, int32_t members, const float *X, int32_t B,
                                       const float *y_mean, const float *y_std, float *Y, float *disagreement,
                                       void *hip_stream);

/* C[M][N] (float32, row stride ldc) = A B with bfloat16 operands (uint16_t
 * bit patterns): A is M x K, stored A[m*lda + k] (a_trans = 0) or
 * A[k*lda + m] (a_trans = 1); B is K x N, stored B[n*ldb + k] (b_trans = 0)
 * or B[k*ldb + n] (b_trans = 1).  Device pointers; enqueued on hip_stream. */
int siminf_gemm_bf16(int32_t M, int32_t N, int32_t K, const uint16_t *A, int32_t lda, int32_t a_trans,
                     const uint16_t *B, int32_t ldb, int32_t b_trans, float *C, int32_t ldc, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* SIMINF_H */
