/*
 * siminf_oracle.c -- plain CPU oracle for the split-step direct-method SSA of
 * Widgren, Bauer, Eriksson & Engblom, "SimInf: An R package for data-driven
 * stochastic disease spread simulations" (arXiv 1605.01421).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the GPU library is checked against.  It shares no source
 * with the GPU library (no headers, helpers, tables or constants): every
 * formula below is written out here from the paper and from the published
 * definitions it names.  Only tests, the smoke check and the CPU-baseline leg
 * of the benchmark may load it.
 *
 * What it computes (per run):
 *   - the per-node continuous-time Markov chain dX = S mu(dt) of section 2.1
 *     (eqs. vectorJSDE and eventupdate), simulated by Gillespie's direct
 *     method exactly as the pseudo-code of Appendix A lays it out: all rates
 *     at the start, then per node and per unit of time the loop
 *     "sum rates -> exponential waiting time -> stop at the day boundary ->
 *     inversion search -> add column S[,n] -> recompute rates flagged by G";
 *   - the scheduled events of section 3.3 (exit, enter, internal transfer in
 *     the node's own thread = E1; external transfer serially afterwards = E2),
 *     same-time order exit < enter < internal < external (section 3.3);
 *   - the post-time-step callback (section 3.4.1, eq. numstep3) once per node
 *     per unit of time after E1 and E2;
 *   - recording of U and V whenever time passes a tspan point (Table 1).
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11,
 * "Parallel random numbers: as easy as 1, 2, 3") used as a keyed counter
 * function, so every draw is fixed by (seed, stream, node, day, draw index)
 * and the result does not depend on the thread count.
 *
 * Floating point: IEEE binary64, round to nearest, no contraction
 * (compiled with -ffp-contract=off), no library log: the exponential
 * variate uses the documented atanh-series logarithm `plog` below.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- status codes (negative = error) ---------------------------------- */
#define OR_OK 0
#define OR_E_ARG (-1)
#define OR_E_UNSUPPORTED (-2)
#define OR_E_ALLOC (-3)
#define OR_E_NEG_STATE (-5)
#define OR_E_BAD_RATE (-6)
#define OR_E_EVENT_OVERDRAW (-7)
#define OR_E_EVENT_INDEX (-8)
#define OR_E_PTS (-9)
#define OR_E_STEP_LIMIT (-10)

/* Implementation limit, not part of the method: the Appendix A loop has no
 * bound on the number of steps a node takes within one unit of time.  Here
 * the draw index k of a node-day is the first Philox counter word, so a
 * node-day owns 2^32 distinct blocks and cannot go past that without
 * repeating draws; the limit is set far below, at 2^24 draws, so that one
 * node with exploding rates ends the run instead of holding it for hours.
 * A node that would need the draw with index OR_STEP_LIMIT (counted from 0)
 * stops the run with OR_E_STEP_LIMIT, keyed like any SSA error (day step,
 * phase SSA, node); the test sits after the lambda test and before the
 * draw, so every node-day that needs at most OR_STEP_LIMIT draws is the
 * method's own result. */
#define OR_STEP_LIMIT (1u << 24)

/* phases of one unit of time, in the order of Appendix A */

#define PH_SSA 0
#define PH_E1 1
#define PH_E2 2
#define PH_PTS 3

/* models with built-in rate functions */
#define MODEL_SIR 0
#define MODEL_SIS 1
#define MODEL_SISE 2
#define MODEL_BIRTH_DEATH 3
#define MODEL_IMMIGRATION_DEATH 4
#define MODEL_SISE_SP 5
/* models given as transition strings (section 5.1): ids from 64 on, their
 * propensities as postfix programs (oracle/mparse.py parses them) */
#define MODEL_GENERATED_FIRST 64

/* event type codes of Table 2 */
#define EV_EXIT 0
#define EV_ENTER 1
#define EV_INTTRANS 2
#define EV_EXTTRANS 3

/* The oracle's own description of one model run.  Layouts follow Table 1:
 * u0 is Nc x Nn column-major (u0[c + i*Nc]); v0 is Nv x Nn; ldata Nld x Nn;
 * S is Nc x Nt and G is Nt x Nt, both column-major; E is Nc x Ecols and
 * N is Nc x Ncols (Table 2).  Event vectors are 0-based; shift < 0 = none. */
typedef struct {
    int32_t model, Nc, Nt, Nn, Nv, Nld, Ngd, Ntspan;
    const int32_t *S, *G, *u0;
    const double *v0, *ldata, *gdata, *tspan;
    int32_t Nev, Ecols, Ncols;
    const int32_t *ev_type, *ev_time, *ev_node, *ev_dest, *ev_n, *ev_select,
        *ev_shift;
    const double *ev_prop;
    const int32_t *E, *N;
    /* SISe_sp: the sparse distance matrix of section 4.2 in compressed
     * columns: node i's neighbours are nb_idx[nb_ptr[i] .. nb_ptr[i+1]),
     * at distances nb_dist (same positions).  Unused by the other models. */
    int32_t Nnb;
    const int32_t *nb_ptr, *nb_idx;
    const double *nb_dist;
    /* generated models: propensity j is the postfix program
     * prog[prog_off[j] .. prog_off[j+1]) over the constants consts[] */
    const int32_t *prog_off, *prog;
    const double *consts;
    int32_t solver; /* SOLVER_SSM or SOLVER_AEM */
} oracle_model;

/* postfix program operations of a generated model's propensity: the low 8
 * bits of a program word, the argument (an index) above them */
#define OP_CONST 0 /* push consts[arg] */
#define OP_U 1     /* push (double)u[arg] */
#define OP_GD 2    /* push gd[arg] */
#define OP_LD 3    /* push ld[arg] */
#define OP_V 4     /* push v[arg] */
#define OP_ADD 5
#define OP_SUB 6
#define OP_MUL 7
#define OP_DIV 8
#define OP_NEG 9

/* ======================================================================
 * Philox4x32-10 (SC'11).  One round maps counter (c0,c1,c2,c3) with key
 * (k0,k1) to (hi(M1*c2)^c1^k0, lo(M1*c2), hi(M0*c0)^c3^k1, lo(M0*c0));
 * the key is bumped by the Weyl constants between rounds; ten rounds.
 * ====================================================================== */
void oracle_philox(const uint32_t key[2], const uint32_t ctr[4],
                   uint32_t out[4]) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t k0 = key[0], k1 = key[1];
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* Uniform on (0,1) from two 32-bit words: k = 52 bits (a's 32 bits on top of
 * b's upper 20 bits); r = (k + 1/2) * 2^-52, exact, never 0 or 1. */
double oracle_uniform(uint32_t a, uint32_t b) {
    uint64_t k = ((uint64_t)a << 20) | (uint64_t)(b >> 12);
    return ((double)k + 0.5) * 0x1p-52;
}

/* Natural logarithm for x in (0, 1] (normal numbers), written out so that
 * every operation is one IEEE rounding:
 *   x = m * 2^e with m in [1,2) taken from the bit pattern;
 *   if m > sqrt(2): m = m/2, e = e+1        (so m in (sqrt(1/2), sqrt(2)])
 *   s = (m-1)/(m+1);  z = s*s
 *   ln m = 2*atanh(s) = 2s * sum_{k=0..11} z^k/(2k+1)
 *          (Horner in z, each step p*z + c one fused multiply-add)
 *   ln x = fma(e, LN2_HI, fma(e, LN2_LO, ln m))
 * with LN2_HI/LN2_LO the classic two-part split of ln 2 (upper part with
 * 32 trailing zero bits so e*LN2_HI is exact).  Series truncation < 2^-60
 * relative since |s| <= 0.1716.  fma() is the C library's correctly rounded
 * fused multiply-add; the clone for processors with FMA instructions
 * computes the same values. */
__attribute__((target_clones("fma", "default")))
double oracle_plog(double x) {
    const double SQRT2 = 0x1.6a09e667f3bcdp+0;
    const double LN2_HI = 0x1.62e42feep-1;
    const double LN2_LO = 0x1.a39ef35793c76p-33;
    uint64_t bits;
    memcpy(&bits, &x, sizeof bits);
    int e = (int)((bits >> 52) & 0x7ff) - 1023;
    uint64_t mbits = (bits & 0x000fffffffffffffull) | 0x3ff0000000000000ull;
    double m;
    memcpy(&m, &mbits, sizeof m);
    if (m > SQRT2) {
        m = m * 0.5;
        e = e + 1;
    }
    double f = m - 1.0;
    double s = f / (m + 1.0);
    double z = s * s;
    double p = 1.0 / 23.0;
    p = fma(p, z, 1.0 / 21.0);
    p = fma(p, z, 1.0 / 19.0);
    p = fma(p, z, 1.0 / 17.0);
    p = fma(p, z, 1.0 / 15.0);
    p = fma(p, z, 1.0 / 13.0);
    p = fma(p, z, 1.0 / 11.0);
    p = fma(p, z, 1.0 / 9.0);
    p = fma(p, z, 1.0 / 7.0);
    p = fma(p, z, 1.0 / 5.0);
    p = fma(p, z, 1.0 / 3.0);
    p = fma(p, z, 1.0);
    double lnm = (s + s) * p;
    double de = (double)e;
    return fma(de, LN2_HI, fma(de, LN2_LO, lnm));
}

/* ---- RNG keying --------------------------------------------------------
 * key = (seed low word, seed high word)
 * SSA step k of node i while simulating towards day boundary T:
 *     counter = (k, (uint32)T, i, (stream & 0xFFFFFF) | 0<<24)
 * event sampling, block b of the event with input index e:
 *     counter = (b, 0, e, (stream & 0xFFFFFF) | 1<<24)            */
#define PURPOSE_SSA 0u
#define PURPOSE_EVENT 1u
#define PURPOSE_AEM 2u /* the all events method's per-channel streams */

/* solvers (section 3.4): the split-step direct method, and the all events
 * method, whose transition channels each draw from a private stream */
#define SOLVER_SSM 0
#define SOLVER_AEM 1

typedef struct {
    uint32_t key[2];
    uint32_t ctr[4];
    uint32_t buf[4];
    int used; /* words of buf already consumed (4 = refill) */
} word_stream;

static void ws_init(word_stream *w, uint64_t seed, uint32_t stream,
                    uint32_t event_index) {
    w->key[0] = (uint32_t)seed;
    w->key[1] = (uint32_t)(seed >> 32);
    w->ctr[0] = 0;
    w->ctr[1] = 0;
    w->ctr[2] = event_index;
    w->ctr[3] = (stream & 0xFFFFFFu) | (PURPOSE_EVENT << 24);
    w->used = 4;
}

static uint32_t ws_next(word_stream *w) {
    if (w->used == 4) {
        oracle_philox(w->key, w->ctr, w->buf);
        w->ctr[0] += 1;
        w->used = 0;
    }
    return w->buf[w->used++];
}

/* Unbiased integer in [0, R), R >= 1: Lemire's multiply-and-reject
 * ("Fast random integer generation in an interval", ACM TOMACS 2019). */
static uint32_t ws_bounded(word_stream *w, uint32_t R) {
    uint64_t m = (uint64_t)ws_next(w) * (uint64_t)R;
    uint32_t l = (uint32_t)m;
    if (l < R) {
        uint32_t t = (uint32_t)(0u - R) % R;
        while (l < t) {
            m = (uint64_t)ws_next(w) * (uint64_t)R;
            l = (uint32_t)m;
        }
    }
    return (uint32_t)(m >> 32);
}

/* ======================================================================
 * Built-in transition-rate functions (the TRFun of section 3.4.1) and
 * post-time-step functions (PTSFun).  Operation order is normative.
 * ====================================================================== */

/* rate of transition j for node state u, continuous state v, local data
 * ld and global data gd. */
static double rate_fn(int model, int j, const int32_t *u, const double *v,
                      const double *ld, const double *gd) {
    (void)ld;
    switch (model) {
    case MODEL_SIR: {
        /* eq. SIR: S -> I at beta*S*I/(S+I+R) (0 for an empty node),
         * I -> R at gamma*I; the listing of Appendix C gives the order. */
        double S = (double)u[0], I = (double)u[1], R = (double)u[2];
        if (j == 0) {
            double n = (S + I) + R;
            if (n > 0.0)
                return ((gd[0] * S) * I) / n;
            return 0.0;
        }
        return gd[1] * I;
    }
    case MODEL_SIS: {
        /* eqs. sirtrans/SIRstoich: S+I -> 2I at beta*S*I, I -> S at gamma*I */
        double S = (double)u[0], I = (double)u[1];
        if (j == 0)
            return (gd[0] * S) * I;
        return gd[1] * I;
    }
    case MODEL_SISE:
    case MODEL_SISE_SP: {
        /* eq. vtectrans: S -> I at upsilon*phi per susceptible,
         * I -> S at gamma per infected. gdata = (upsilon, gamma, ...). */
        double S = (double)u[0], I = (double)u[1];
        if (j == 0)
            return (gd[0] * v[0]) * S;
        return gd[1] * I;
    }
    case MODEL_BIRTH_DEATH: {
        /* X -> 2X at b*X, X -> 0 at d*X; gdata = (b, d) */
        double X = (double)u[0];
        if (j == 0)
            return gd[0] * X;
        return gd[1] * X;
    }
    case MODEL_IMMIGRATION_DEATH: {
        /* 0 -> X at kappa, X -> 0 at mu*X; gdata = (kappa, mu) */
        double X = (double)u[0];
        if (j == 0)
            return gd[0];
        return gd[1] * X;
    }
    }
    return NAN;
}

/* Propensity j of a generated model: its postfix program run on a stack of
 * binary64 values, one IEEE operation per operator (operands left, then
 * right).  A malformed program gives NaN, which the caller reports as a bad
 * rate. */
static double rate_gen(const oracle_model *m, int j, const int32_t *u, const double *v,
                       const double *ld, const double *gd) {
    double st[64];
    int sp = 0;
    for (int k = m->prog_off[j]; k < m->prog_off[j + 1]; ++k) {
        int op = m->prog[k] & 0xff, arg = m->prog[k] >> 8;
        if (op <= OP_V) {
            if (sp >= 64)
                return NAN;
            st[sp++] = op == OP_CONST ? m->consts[arg]
                       : op == OP_U   ? (double)u[arg]
                       : op == OP_GD  ? gd[arg]
                       : op == OP_LD  ? ld[arg]
                                      : v[arg];
        } else if (op == OP_NEG) {
            if (sp < 1)
                return NAN;
            st[sp - 1] = -st[sp - 1];
        } else {
            if (sp < 2)
                return NAN;
            double a = st[sp - 2], b = st[sp - 1];
            sp -= 1;
            st[sp - 1] = op == OP_ADD ? a + b : op == OP_SUB ? a - b : op == OP_MUL ? a * b : a / b;
        }
    }
    return sp == 1 ? st[0] : NAN;
}

static double rate_any(const oracle_model *m, int j, const int32_t *u, const double *v,
                       const double *ld, const double *gd) {
    if (m->model >= MODEL_GENERATED_FIRST)
        return rate_gen(m, j, u, v, ld, gd);
    return rate_fn(m->model, j, u, v, ld, gd);
}

static int model_dims(int model, int *Nc, int *Nt, int *Nv, int *Nld,
                      int *Ngd) {
    switch (model) {
    case MODEL_SIR:
        *Nc = 3; *Nt = 2; *Nv = 0; *Nld = 0; *Ngd = 2;
        return 1;
    case MODEL_SIS:
        *Nc = 2; *Nt = 2; *Nv = 0; *Nld = 0; *Ngd = 2;
        return 1;
    case MODEL_SISE:
        *Nc = 2; *Nt = 2; *Nv = 1; *Nld = 4; *Ngd = 7;
        return 1;
    case MODEL_SISE_SP:
        *Nc = 2; *Nt = 2; *Nv = 1; *Nld = 4; *Ngd = 8;
        return 1;
    case MODEL_BIRTH_DEATH:
    case MODEL_IMMIGRATION_DEATH:
        *Nc = 1; *Nt = 2; *Nv = 0; *Nld = 0; *Ngd = 2;
        return 1;
    }
    return 0;
}

/* Day of year of integer day T (1..365), T = 1 is day 1. */
static int day_of_year(int64_t T) {
    int64_t r = (T - 1) % 365;
    if (r < 0)
        r += 365;
    return (int)r + 1;
}

/* Post-time-step function: returns 0 or a negative error. v_new gets the
 * new continuous state.  SISe: one explicit-Euler step of unit length of
 * d phi/dt = alpha*I/N - beta(t)*phi (eq. envInfPressure-local-spread with
 * no spatial coupling), i.e. phi' = phi*(1-beta_q) + alpha*I/N, where the
 * season q is the first k with day-of-year <= end_k (ldata), else season 0;
 * I/N is taken as 0 for an empty node. */
/* SISe_sp (section 4.2, eq. envInfPressure-local-spread): one explicit-
 * Euler step of unit length of
 *   d phi_i/dt = alpha I_i/N_i + sum_k (phi_k N_k - phi_i N_i)/N_i * D/d_ik
 *                - beta(t) phi_i
 * taken, in this order, as
 *   phi_i' = (phi_i (1 - beta_q) + alpha I_i / N_i) + c_i,
 *   c_i = sum over the neighbours k in stored order of
 *         ((phi_k N_k - phi_i N_i) / N_i) * (D / d_ik),
 * with every phi the value before this step (all nodes are advanced from
 * the same state) and N = S + I after the day's events; the alpha and the
 * coupling terms are 0 for an empty node.  D = gdata[7]. */
static int pts_sise_sp(const oracle_model *m, double *v_new, const int32_t *u, const double *v, int i,
                       int64_t T) {
    const double *ld = m->ldata + (size_t)i * m->Nld;
    const double *gd = m->gdata;
    const int32_t *ui = u + (size_t)i * 2;
    int doy = day_of_year(T);
    int q = 0;
    for (int k = 3; k >= 0; --k)
        if ((double)doy <= ld[k])
            q = k;
    double beta = gd[3 + q];
    double a = v[i] * (1.0 - beta);
    int32_t Ni = ui[0] + ui[1];
    double b = 0.0;
    double c = 0.0;
    if (Ni > 0) {
        b = (gd[2] * (double)ui[1]) / (double)Ni;
        for (int e = m->nb_ptr[i]; e < m->nb_ptr[i + 1]; ++e) {
            int k = m->nb_idx[e];
            int32_t Nk = u[(size_t)k * 2] + u[(size_t)k * 2 + 1];
            double flow = (v[k] * (double)Nk) - (v[i] * (double)Ni);
            double term = (flow / (double)Ni) * (gd[7] / m->nb_dist[e]);
            c = c + term;
        }
    }
    double phi = (a + b) + c;
    if (!isfinite(phi))
        return OR_E_PTS;
    v_new[0] = phi;
    return 0;
}

static int pts_fn(int model, double *v_new, const int32_t *u, const double *v,
                  const double *ld, const double *gd, int Nv, int64_t T) {
    if (model == MODEL_SISE) {
        int doy = day_of_year(T);
        int q = 0;
        for (int k = 3; k >= 0; --k)
            if ((double)doy <= ld[k])
                q = k;
        double beta = gd[3 + q];
        double a = v[0] * (1.0 - beta);
        int32_t Nn = u[0] + u[1];
        double b = 0.0;
        if (Nn > 0)
            b = (gd[2] * (double)u[1]) / (double)Nn;
        double phi = a + b;
        if (!isfinite(phi))
            return OR_E_PTS;
        v_new[0] = phi;
        return 0;
    }
    for (int k = 0; k < Nv; ++k)
        v_new[k] = v[k];
    return 0;
}

/* The k-th unit exponential of channel j of node i (all events method):
 * -log of the uniform from the first two words of the Philox block
 * (k, j, i, stream | PURPOSE_AEM << 24). */
static double aem_exp(uint64_t seed, uint32_t stream, int i, int j, uint32_t k) {
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {k, (uint32_t)j, (uint32_t)i, (stream & 0xFFFFFFu) | (PURPOSE_AEM << 24)};
    uint32_t r[4];
    oracle_philox(key, ctr, r);
    return -oracle_plog(oracle_uniform(r[0], r[1]));
}

/* ---- error keys ------------------------------------------------------
 * (boundary index, phase, index) ordered lexicographically, packed into a
 * 64-bit key so that the smallest key is the first error in the serial
 * order of Appendix A; the code sits in the low 4 bits. */
static uint64_t make_key(int64_t b, int phase, int64_t index, int code) {
    return ((uint64_t)b << 40) | ((uint64_t)phase << 36) |
           ((uint64_t)(uint32_t)index << 4) | (uint64_t)(-code);
}

/* ---- one scheduled event (section 3.3) ------------------------------- */
/* Applies event e to node state u (and dest state ud for an external
 * transfer).  Returns 0 or a negative error code; on error the states are
 * left unchanged. */
static int apply_event(const oracle_model *m, int e, int32_t *u, int32_t *ud,
                       uint64_t seed, uint32_t stream) {
    const int Nc = m->Nc;
    int type = m->ev_type[e];
    int s = m->ev_select[e];
    if (s < 0 || s >= m->Ecols)
        return OR_E_EVENT_INDEX;
    const int32_t *Ecol = m->E + (size_t)s * Nc;
    if (type == EV_ENTER) {
        /* n individuals into the first compartment selected by E[,s] */
        for (int c = 0; c < Nc; ++c)
            if (Ecol[c] != 0) {
                if (m->ev_n[e] < 0)
                    return OR_E_EVENT_INDEX;
                u[c] += m->ev_n[e];
                return 0;
            }
        return OR_E_EVENT_INDEX;
    }
    /* shift targets (Table 2): individual in compartment p goes to
     * p + N[p,q]; no shift leaves them in p. */
    int q = m->ev_shift[e];
    int target[64];
    if (q >= m->Ncols)
        return OR_E_EVENT_INDEX;
    for (int c = 0; c < Nc; ++c) {
        target[c] = c;
        if (q >= 0)
            target[c] = c + m->N[(size_t)q * Nc + c];
        if (Ecol[c] != 0 && (target[c] < 0 || target[c] >= Nc))
            return OR_E_EVENT_INDEX;
    }
    int64_t tot = 0;
    for (int c = 0; c < Nc; ++c)
        if (Ecol[c] != 0)
            tot += u[c];
    int64_t n = m->ev_n[e];
    if (n < 0)
        return OR_E_EVENT_INDEX;
    if (n == 0) {
        /* proportion of the selected total, rounded half away from zero */
        double x = m->ev_prop[e] * (double)tot;
        n = (int64_t)floor(x + 0.5);
    }
    if (n > tot)
        return OR_E_EVENT_OVERDRAW;
    int32_t take[64];
    for (int c = 0; c < Nc; ++c)
        take[c] = 0;
    if (n == tot) {
        for (int c = 0; c < Nc; ++c)
            if (Ecol[c] != 0)
                take[c] = u[c];
    } else {
        /* individual-by-individual sampling without replacement from the
         * pooled selected compartments: draw j uniform in [0, remaining),
         * the individual belongs to the first compartment whose running
         * count of not-yet-drawn individuals exceeds j. */
        word_stream w;
        ws_init(&w, seed, stream, (uint32_t)e);
        for (int64_t k = 0; k < n; ++k) {
            uint32_t j = ws_bounded(&w, (uint32_t)(tot - k));
            int64_t run = 0;
            for (int c = 0; c < Nc; ++c) {
                if (Ecol[c] == 0)
                    continue;
                run += u[c] - take[c];
                if ((int64_t)j < run) {
                    take[c] += 1;
                    break;
                }
            }
        }
    }
    for (int c = 0; c < Nc; ++c)
        u[c] -= take[c];
    if (type == EV_EXIT)
        return 0;
    int32_t *dst = (type == EV_EXTTRANS) ? ud : u;
    for (int c = 0; c < Nc; ++c)
        dst[target[c]] += take[c];
    return 0;
}

/* ---- event order: (time, type, input index) --------------------------- */
static const oracle_model *g_sort_model;
static int cmp_events(const void *pa, const void *pb) {
    int a = *(const int *)pa, b = *(const int *)pb;
    const oracle_model *m = g_sort_model;
    if (m->ev_time[a] != m->ev_time[b])
        return m->ev_time[a] < m->ev_time[b] ? -1 : 1;
    if (m->ev_type[a] != m->ev_type[b])
        return m->ev_type[a] < m->ev_type[b] ? -1 : 1;
    return a < b ? -1 : (a > b);
}

/* ======================================================================
 * oracle_run: one trajectory.  U (Nc*Nn x Ntspan, column-major) and V
 * (Nv*Nn x Ntspan) are filled for every recorded tspan point.  counters
 * = {transitions, node-days, events applied}.  err = {code, boundary
 * index, phase, index}.  Returns 0 or the first error's code.
 * ====================================================================== */
int oracle_run(const oracle_model *m, uint64_t seed, uint32_t stream,
               int nthreads, int32_t *U, double *V, uint64_t *counters,
               int64_t *err) {
    int Nc, Nt, Nv, Nld, Ngd;
    err[0] = 0;
    err[1] = err[2] = err[3] = -1;
    counters[0] = counters[1] = counters[2] = 0;
    if (m->solver != SOLVER_SSM && m->solver != SOLVER_AEM)
        return err[0] = OR_E_ARG;
    if (m->model >= MODEL_GENERATED_FIRST) {
        /* a generated model has the sizes it was given */
        if (!m->prog_off || !m->prog || m->Nc < 1 || m->Nt < 1 || m->Nt > 32 || m->Nv > 64)
            return err[0] = OR_E_ARG;
        Nc = m->Nc; Nt = m->Nt; Nv = m->Nv; Nld = m->Nld; Ngd = m->Ngd;
    } else if (!model_dims(m->model, &Nc, &Nt, &Nv, &Nld, &Ngd))
        return err[0] = OR_E_UNSUPPORTED;
    if (m->Nc != Nc || m->Nt != Nt || m->Nv != Nv || m->Nld < Nld ||
        m->Ngd < Ngd || m->Nn < 0 || m->Ntspan < 1 || m->Nev < 0)
        return err[0] = OR_E_ARG;
    const int Nn = m->Nn;
    const int Ntspan = m->Ntspan;
    if (m->model == MODEL_SISE_SP) {
        /* the neighbour lists: within the nodes, positive finite distances */
        if (!m->nb_ptr || (m->Nnb > 0 && (!m->nb_idx || !m->nb_dist)) || m->nb_ptr[0] != 0 ||
            m->nb_ptr[Nn] != m->Nnb)
            return err[0] = OR_E_ARG;
        for (int i = 0; i < Nn; ++i)
            if (m->nb_ptr[i + 1] < m->nb_ptr[i])
                return err[0] = OR_E_ARG;
        for (int e = 0; e < m->Nnb; ++e)
            if (m->nb_idx[e] < 0 || m->nb_idx[e] >= Nn || !(m->nb_dist[e] > 0.0) || !isfinite(m->nb_dist[e]))
                return err[0] = OR_E_ARG;
    }
    for (int k = 1; k < Ntspan; ++k)
        if (!(m->tspan[k] > m->tspan[k - 1]))
            return err[0] = OR_E_ARG;
    if (nthreads < 1)
        nthreads = 1;

    int32_t *u = malloc(sizeof(int32_t) * (size_t)Nc * (Nn ? Nn : 1));
    double *v = malloc(sizeof(double) * (size_t)(Nv ? Nv : 1) * (Nn ? Nn : 1));
    double *v_next = malloc(sizeof(double) * (size_t)(Nv ? Nv : 1) * (Nn ? Nn : 1));
    int *order = malloc(sizeof(int) * (size_t)(m->Nev ? m->Nev : 1));
    int *e1_start = calloc((size_t)Nn + 1, sizeof(int));
    int *e1_list = malloc(sizeof(int) * (size_t)(m->Nev ? m->Nev : 1));
    int *e1_cursor = calloc((size_t)(Nn ? Nn : 1), sizeof(int));
    int *e2_list = malloc(sizeof(int) * (size_t)(m->Nev ? m->Nev : 1));
    uint64_t *node_err = malloc(sizeof(uint64_t) * (size_t)(Nn ? Nn : 1));
    uint64_t *node_trans = calloc((size_t)(Nn ? Nn : 1), sizeof(uint64_t));
    uint64_t *node_events = calloc((size_t)(Nn ? Nn : 1), sizeof(uint64_t));
    /* all events method: per node and channel the integrated rate, the
     * next firing level and the index of the next exponential */
    const size_t nch = (size_t)(Nn ? Nn : 1) * (size_t)Nt;
    double *aem_T = m->solver == SOLVER_AEM ? calloc(nch, sizeof(double)) : NULL;
    double *aem_P = m->solver == SOLVER_AEM ? malloc(nch * sizeof(double)) : NULL;
    uint32_t *aem_K = m->solver == SOLVER_AEM ? malloc(nch * sizeof(uint32_t)) : NULL;
    if (!u || !v || !v_next || !order || !e1_start || !e1_list || !e1_cursor ||
        !e2_list || !node_err || !node_trans || !node_events ||
        (m->solver == SOLVER_AEM && (!aem_T || !aem_P || !aem_K))) {
        free(u); free(v); free(v_next); free(order); free(e1_start); free(e1_list);
        free(e1_cursor); free(e2_list); free(node_err); free(node_trans);
        free(node_events); free(aem_T); free(aem_P); free(aem_K);
        return err[0] = OR_E_ALLOC;
    }
    if (m->solver == SOLVER_AEM)
        for (int i = 0; i < Nn; ++i)
            for (int j = 0; j < Nt; ++j) {
                aem_P[(size_t)i * Nt + j] = aem_exp(seed, stream, i, j, 0);
                aem_K[(size_t)i * Nt + j] = 1;
            }
    memcpy(u, m->u0, sizeof(int32_t) * (size_t)Nc * Nn);
    if (Nv)
        memcpy(v, m->v0, sizeof(double) * (size_t)Nv * Nn);

    /* events: sort by (time, type, input index); split into per-node E1
     * lists (each in that order) and one E2 list. */
    int bad_event = -1;
    for (int e = 0; e < m->Nev; ++e) {
        order[e] = e;
        int ty = m->ev_type[e];
        if (ty < EV_EXIT || ty > EV_EXTTRANS || m->ev_node[e] < 0 ||
            m->ev_node[e] >= Nn ||
            (ty == EV_EXTTRANS && (m->ev_dest[e] < 0 || m->ev_dest[e] >= Nn)))
            if (bad_event < 0)
                bad_event = e;
    }
    if (bad_event >= 0) {
        err[0] = OR_E_EVENT_INDEX;
        err[3] = bad_event;
        goto done;
    }
    g_sort_model = m;
    qsort(order, (size_t)m->Nev, sizeof(int), cmp_events);
    int n_e2 = 0;
    for (int k = 0; k < m->Nev; ++k) {
        int e = order[k];
        if (m->ev_type[e] == EV_EXTTRANS)
            e2_list[n_e2++] = e;
        else
            e1_start[m->ev_node[e] + 1] += 1;
    }
    for (int i = 0; i < Nn; ++i)
        e1_start[i + 1] += e1_start[i];
    for (int i = 0; i < Nn; ++i)
        e1_cursor[i] = e1_start[i];
    for (int k = 0; k < m->Nev; ++k) {
        int e = order[k];
        if (m->ev_type[e] != EV_EXTTRANS)
            e1_list[e1_cursor[m->ev_node[e]]++] = e;
    }
    for (int i = 0; i < Nn; ++i)
        e1_cursor[i] = e1_start[i];
    int e2_cursor = 0;

    /* record every tspan point not after the start time */
    const double t0 = m->tspan[0];
    const double Tend = m->tspan[Ntspan - 1];
    int rec = 0;
    while (rec < Ntspan && m->tspan[rec] <= t0) {
        memcpy(U + (size_t)rec * Nn * Nc, u, sizeof(int32_t) * (size_t)Nc * Nn);
        if (Nv)
            memcpy(V + (size_t)rec * Nn * Nv, v, sizeof(double) * (size_t)Nv * Nn);
        ++rec;
    }

    double t = t0;
    int64_t Tint = (int64_t)floor(t0) + 1;
    int64_t b = 0;
    uint64_t node_days = 0;
    const uint64_t NOERR = UINT64_MAX;

    while (t < Tend) {
        const double T = (double)Tint;
        const uint32_t Tword = (uint32_t)(int32_t)Tint;
        uint64_t phase_err = NOERR;

        /* ---- SSA to T, then this node's E1 events (Appendix A) -------- */
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
        for (int i = 0; i < Nn; ++i) {
            int32_t *ui = u + (size_t)i * Nc;
            const double *vi = v + (size_t)i * Nv;
            const double *ld = m->ldata + (size_t)i * m->Nld;
            double w[32];
            node_err[i] = NOERR;
            int bad = 0;
            for (int j = 0; j < Nt; ++j) {
                w[j] = rate_any(m, j, ui, vi, ld, m->gdata);
                if (!(w[j] >= 0.0) || !isfinite(w[j]))
                    bad = 1;
            }
            if (bad) {
                node_err[i] = make_key(b, PH_SSA, i, OR_E_BAD_RATE);
                continue;
            }
            double ti = t;
            if (m->solver == SOLVER_AEM) {
                /* All events method (section 3.4): channel j fires when its
                 * integrated rate Tj reaches Pj, the running sum of the unit
                 * exponentials of its private stream.  The next channel is
                 * the one with the least (Pj - Tj)/wj (the lowest j on a
                 * tie); the others' integrals advance by wk tau, the fired
                 * one's becomes Pj and Pj takes its next exponential.  At
                 * the day boundary every integral advances to T; the
                 * integrals and sums carry over to the next day. */
                double *Ti = aem_T + (size_t)i * Nt, *Pi = aem_P + (size_t)i * Nt;
                uint32_t *Ki = aem_K + (size_t)i * Nt;
                uint32_t k = 0;
                for (;;) {
                    int n = -1;
                    double best = 0.0;
                    for (int j = 0; j < Nt; ++j) {
                        if (w[j] > 0.0) {
                            double tau = (Pi[j] - Ti[j]) / w[j];
                            if (n < 0 || tau < best) {
                                best = tau;
                                n = j;
                            }
                        }
                    }
                    if (n < 0)
                        break; /* no positive rate: the integrals stay */
                    if (k == OR_STEP_LIMIT) {
                        bad = OR_E_STEP_LIMIT;
                        break;
                    }
                    k++;
                    double tn = ti + best;
                    if (tn >= T) {
                        double rest = T - ti;
                        for (int j = 0; j < Nt; ++j)
                            Ti[j] = Ti[j] + w[j] * rest;
                        break;
                    }
                    for (int j = 0; j < Nt; ++j)
                        if (j != n)
                            Ti[j] = Ti[j] + w[j] * best;
                    Ti[n] = Pi[n];
                    Pi[n] = Pi[n] + aem_exp(seed, stream, i, n, Ki[n]);
                    Ki[n] += 1;
                    ti = tn;
                    for (int c = 0; c < Nc; ++c) {
                        ui[c] += m->S[(size_t)n * Nc + c];
                        if (ui[c] < 0)
                            bad = OR_E_NEG_STATE;
                    }
                    node_trans[i] += 1;
                    if (bad)
                        break;
                    for (int j = 0; j < Nt; ++j) {
                        if (m->G[(size_t)n * Nt + j] != 0) {
                            w[j] = rate_any(m, j, ui, vi, ld, m->gdata);
                            if (!(w[j] >= 0.0) || !isfinite(w[j]))
                                bad = OR_E_BAD_RATE;
                        }
                    }
                    if (bad)
                        break;
                }
            } else {
            uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
            uint32_t ctr[4] = {0, Tword, (uint32_t)i,
                               (stream & 0xFFFFFFu) | (PURPOSE_SSA << 24)};
            uint32_t k = 0;
            for (;;) {
                double lambda = 0.0;
                for (int j = 0; j < Nt; ++j)
                    lambda = lambda + w[j];
                if (!(lambda > 0.0))
                    break; /* nothing can happen: time moves to T */
                if (k == OR_STEP_LIMIT) {
                    bad = OR_E_STEP_LIMIT;
                    break;
                }
                uint32_t r[4];
                ctr[0] = k++;
                oracle_philox(key, ctr, r);
                double r1 = oracle_uniform(r[0], r[1]);
                double r2 = oracle_uniform(r[2], r[3]);
                double tau = (-oracle_plog(r1)) / lambda;
                double tn = ti + tau;
                if (tn >= T)
                    break; /* the step would cross the day boundary */
                ti = tn;
                /* inversion: first n with lambda*r2 <= cumulative sum */
                double x = lambda * r2;
                double cum = 0.0;
                int n = -1, last = -1;
                for (int j = 0; j < Nt; ++j) {
                    cum = cum + w[j];
                    if (w[j] > 0.0) {
                        last = j;
                        if (x <= cum) {
                            n = j;
                            break;
                        }
                    }
                }
                if (n < 0)
                    n = last;
                for (int c = 0; c < Nc; ++c) {
                    ui[c] += m->S[(size_t)n * Nc + c];
                    if (ui[c] < 0)
                        bad = OR_E_NEG_STATE;
                }
                node_trans[i] += 1;
                if (bad)
                    break;
                for (int j = 0; j < Nt; ++j) {
                    if (m->G[(size_t)n * Nt + j] != 0) {
                        w[j] = rate_any(m, j, ui, vi, ld, m->gdata);
                        if (!(w[j] >= 0.0) || !isfinite(w[j]))
                            bad = OR_E_BAD_RATE;
                    }
                }
                if (bad)
                    break;
            }
            }
            if (bad) {
                node_err[i] = make_key(b, PH_SSA, i, bad);
                continue;
            }
            /* E1 events of node i with time <= T, in key order */
            while (e1_cursor[i] < e1_start[i + 1]) {
                int e = e1_list[e1_cursor[i]];
                if ((double)m->ev_time[e] > T)
                    break;
                int rc = apply_event(m, e, ui, NULL, seed, stream);
                if (rc != 0) {
                    node_err[i] = make_key(b, PH_E1, e, rc);
                    break;
                }
                node_events[i] += 1;
                e1_cursor[i] += 1;
            }
        }
        for (int i = 0; i < Nn; ++i)
            if (node_err[i] < phase_err)
                phase_err = node_err[i];
        node_days += (uint64_t)Nn;
        if (phase_err != NOERR)
            goto fail;

        /* ---- E2: external transfers, serially in key order (Appendix A) */
        while (e2_cursor < n_e2) {
            int e = e2_list[e2_cursor];
            if ((double)m->ev_time[e] > T)
                break;
            int rc = apply_event(m, e, u + (size_t)m->ev_node[e] * Nc,
                                 u + (size_t)m->ev_dest[e] * Nc, seed, stream);
            if (rc != 0) {
                phase_err = make_key(b, PH_E2, e, rc);
                goto fail;
            }
            counters[2] += 1;
            e2_cursor += 1;
        }

        /* ---- post time step (Appendix A) ------------------------------- */
        if (m->model == MODEL_SISE_SP) {
            /* every node's step reads its neighbours' values before the
             * step: new values go to a second buffer first */
#pragma omp parallel for schedule(static) num_threads(nthreads)
            for (int i = 0; i < Nn; ++i) {
                node_err[i] = NOERR;
                if (pts_sise_sp(m, v_next + i, u, v, i, Tint) < 0) {
                    node_err[i] = make_key(b, PH_PTS, i, OR_E_PTS);
                    v_next[i] = v[i];
                }
            }
            memcpy(v, v_next, sizeof(double) * (size_t)Nn);
        } else {
#pragma omp parallel for schedule(static) num_threads(nthreads)
            for (int i = 0; i < Nn; ++i) {
                double vnew[64];
                node_err[i] = NOERR;
                int rc = pts_fn(m->model, vnew, u + (size_t)i * Nc,
                                v + (size_t)i * Nv, m->ldata + (size_t)i * m->Nld,
                                m->gdata, Nv, Tint);
                if (rc < 0) {
                    node_err[i] = make_key(b, PH_PTS, i, OR_E_PTS);
                    continue;
                }
                for (int k = 0; k < Nv; ++k)
                    v[(size_t)i * Nv + k] = vnew[k];
            }
        }
        for (int i = 0; i < Nn; ++i)
            if (node_err[i] < phase_err)
                phase_err = node_err[i];
        if (phase_err != NOERR)
            goto fail;

        /* ---- record every tspan point passed (Table 1, U and V) -------- */
        while (rec < Ntspan && m->tspan[rec] <= T) {
            memcpy(U + (size_t)rec * Nn * Nc, u,
                   sizeof(int32_t) * (size_t)Nc * Nn);
            if (Nv)
                memcpy(V + (size_t)rec * Nn * Nv, v,
                       sizeof(double) * (size_t)Nv * Nn);
            ++rec;
        }
        t = T;
        Tint += 1;
        b += 1;
        continue;
    fail:
        err[0] = -(int64_t)(phase_err & 0xF);
        err[1] = (int64_t)(phase_err >> 40);
        err[2] = (int64_t)((phase_err >> 36) & 0xF);
        err[3] = (int64_t)((phase_err >> 4) & 0xFFFFFFFFu);
        break;
    }
    counters[1] = node_days;
    for (int i = 0; i < Nn; ++i) {
        counters[0] += node_trans[i];
        counters[2] += node_events[i];
    }
done:
    free(u); free(v); free(v_next); free(order); free(e1_start); free(e1_list);
    free(e1_cursor); free(e2_list); free(node_err); free(node_trans);
    free(node_events);
    free(aem_T);
    free(aem_P);
    free(aem_K);
    return (int)err[0];
}

/* Number of threads OpenMP would use by default (for reporting). */
int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
