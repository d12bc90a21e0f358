// models.h -- built-in transition-rate and post-time-step functions, one
// functor per model (the TRFun / PTSFun pairs of section 3.4.1).  Device code
// cannot call host function pointers, so each model is a compile-time type
// and the kernels are instantiated per model.  Operation order is normative:
// the results must be bit-identical to any other implementation following
// the same formulas in IEEE binary64.
#pragma once
#include "device_types.h"

namespace siminf {

enum ModelId { M_SIR = 0, M_SIS = 1, M_SISE = 2, M_BIRTH_DEATH = 3, M_IMMIGRATION_DEATH = 4, M_SISE_SP = 5 };

__device__ __forceinline__ double pick(bool c, double a, double b) { return c ? a : b; }

// SIR (eq. SIR): S -> I at beta S I / (S + I + R), 0 for an empty node
// (Appendix C listing); I -> R at gamma I.  gdata = (beta, gamma).
struct ModelSIR {
    static constexpr int ID = M_SIR, NC = 3, NT = 2, NV = 0, NLD = 0, NGD = 2;
    static constexpr bool COUPLED = false, GENERATED = false;
    template <int J>
    __device__ static __forceinline__ double rate(const int32_t* u, const double*, const double*,
                                                  const double* gd) {
        if constexpr (J == 0) {
            const double s = (double)u[0], i = (double)u[1], r = (double)u[2];
            const double n = (s + i) + r;
            return n > 0.0 ? ((gd[0] * s) * i) / n : 0.0;
        } else {
            return gd[1] * (double)u[1];
        }
    }
    __device__ static __forceinline__ bool pts(double*, const int32_t*, const double*, const double*,
                                               int64_t) {
        return true;
    }
    // the post-time step leaves every state unchanged
    __device__ static __forceinline__ bool pts_fixed(const double*, const int32_t*) { return true; }
};

// SIS (eqs. sirtrans, SIRstoich): S + I -> 2I at beta S I; I -> S at gamma I.
struct ModelSIS {
    static constexpr int ID = M_SIS, NC = 2, NT = 2, NV = 0, NLD = 0, NGD = 2;
    static constexpr bool COUPLED = false, GENERATED = false;
    template <int J>
    __device__ static __forceinline__ double rate(const int32_t* u, const double*, const double*,
                                                  const double* gd) {
        if constexpr (J == 0)
            return (gd[0] * (double)u[0]) * (double)u[1];
        else
            return gd[1] * (double)u[1];
    }
    __device__ static __forceinline__ bool pts(double*, const int32_t*, const double*, const double*,
                                               int64_t) {
        return true;
    }
    // the post-time step leaves every state unchanged
    __device__ static __forceinline__ bool pts_fixed(const double*, const int32_t*) { return true; }
};

// SISe (section 4.2 without the spatial coupling term): S -> I at upsilon phi
// per susceptible, I -> S at gamma per infected.  After every unit of time
// phi is advanced by one explicit-Euler step of length 1 of
// d phi/dt = alpha I/N - beta(t) phi (eq. numstep3):
//   phi <- phi (1 - beta_q) + alpha I / N,  N = S + I (the I/N term is 0 if N = 0)
// with season q the first of the four whose end day-of-year (ldata) is >= the
// day of year of the new day, else the first season.
// gdata = (upsilon, gamma, alpha, beta_1, beta_2, beta_3, beta_4).
struct ModelSISe {
    static constexpr int ID = M_SISE, NC = 2, NT = 2, NV = 1, NLD = 4, NGD = 7;
    static constexpr bool COUPLED = false, GENERATED = false;
    template <int J>
    __device__ static __forceinline__ double rate(const int32_t* u, const double* v, const double*,
                                                  const double* gd) {
        if constexpr (J == 0)
            return (gd[0] * v[0]) * (double)u[0];
        else
            return gd[1] * (double)u[1];
    }
    __device__ static __forceinline__ bool pts(double* v, const int32_t* u, const double* ld,
                                               const double* gd, int64_t day) {
        // (day - 1) mod 365 in [0, 365); 32-bit arithmetic for the usual days
        const int64_t dm = day - 1;
        int64_t r;
        if (dm >= 0 && dm <= 0x7FFFFFFF) {
            r = (int64_t)((uint32_t)dm % 365u);
        } else {
            r = dm % 365;
            if (r < 0) r += 365;
        }
        const double doy = (double)(r + 1);
        // selects on values (not on array elements) keep the node in registers
        const double decay = pick(doy <= ld[0], gd[3],
                                  pick(doy <= ld[1], gd[4],
                                       pick(doy <= ld[2], gd[5], pick(doy <= ld[3], gd[6], gd[3]))));
        const double kept = v[0] * (1.0 - decay);
        const int32_t total = u[0] + u[1];
        const double shed = total > 0 ? (gd[2] * (double)u[1]) / (double)total : 0.0;
        const double phi = kept + shed;
        v[0] = phi;
        return isfinite(phi);
    }
    // states the post-time step maps to themselves bit for bit: phi = +0 with
    // no infected (kept = +0 (1 - beta) is +0 or -0, shed = +0, the sum +0)
    __device__ static __forceinline__ bool pts_fixed(const double* v, const int32_t* u) {
        return __double_as_longlong(v[0]) == 0 && u[1] == 0;
    }
};

// SISe_sp (section 4.2): SISe with the spatial coupling of the environmental
// pressure among proximal nodes.  The rates are SISe's; the post-time step
// is one explicit-Euler step of unit length of eq.
// envInfPressure-local-spread,
//   phi_i <- (phi_i (1 - beta_q) + alpha I_i / N_i) + c_i,
//   c_i = sum over the neighbours k, in stored order, of
//         ((phi_k N_k - phi_i N_i) / N_i) * w_ik,   w_ik = D / d_ik,
// every phi taken before the step and N = S + I after the day's events; the
// alpha term and c_i are 0 for an empty node.  The kernel gathers c_i from
// the neighbours (coupling_term) and hands it to pts_coupled; only the
// dataflow kernel, where every node is resident, runs this model.
// gdata = (upsilon, gamma, alpha, beta_1, beta_2, beta_3, beta_4, D).
struct ModelSISeSp {
    static constexpr int ID = M_SISE_SP, NC = 2, NT = 2, NV = 1, NLD = 4, NGD = 8;
    static constexpr bool COUPLED = true, GENERATED = false;
    template <int J>
    __device__ static __forceinline__ double rate(const int32_t* u, const double* v, const double* ld,
                                                  const double* gd) {
        return ModelSISe::template rate<J>(u, v, ld, gd);
    }
    __device__ static __forceinline__ double coupling_term(double phi_k, int32_t n_k, double phi_i, int32_t n_i,
                                                           double w) {
        const double flow = (phi_k * (double)n_k) - (phi_i * (double)n_i);
        return (flow / (double)n_i) * w;
    }
    __device__ static __forceinline__ bool pts_coupled(double* v, const int32_t* u, const double* ld,
                                                       const double* gd, int64_t day, double c) {
        const int64_t dm = day - 1;
        int64_t r;
        if (dm >= 0 && dm <= 0x7FFFFFFF) {
            r = (int64_t)((uint32_t)dm % 365u);
        } else {
            r = dm % 365;
            if (r < 0) r += 365;
        }
        const double doy = (double)(r + 1);
        const double decay = pick(doy <= ld[0], gd[3],
                                  pick(doy <= ld[1], gd[4],
                                       pick(doy <= ld[2], gd[5], pick(doy <= ld[3], gd[6], gd[3]))));
        const double kept = v[0] * (1.0 - decay);
        const int32_t total = u[0] + u[1];
        const double shed = total > 0 ? (gd[2] * (double)u[1]) / (double)total : 0.0;
        const double phi = (kept + shed) + c;
        v[0] = phi;
        return isfinite(phi);
    }
    __device__ static __forceinline__ bool pts_fixed(const double*, const int32_t*) { return false; }
};

// Linear birth-death: X -> 2X at b X, X -> 0 at d X.  gdata = (b, d).
struct ModelBirthDeath {
    static constexpr int ID = M_BIRTH_DEATH, NC = 1, NT = 2, NV = 0, NLD = 0, NGD = 2;
    static constexpr bool COUPLED = false, GENERATED = false;
    template <int J>
    __device__ static __forceinline__ double rate(const int32_t* u, const double*, const double*,
                                                  const double* gd) {
        return gd[J] * (double)u[0];
    }
    __device__ static __forceinline__ bool pts(double*, const int32_t*, const double*, const double*,
                                               int64_t) {
        return true;
    }
    // the post-time step leaves every state unchanged
    __device__ static __forceinline__ bool pts_fixed(const double*, const int32_t*) { return true; }
};

// Immigration-death: 0 -> X at kappa, X -> 0 at mu X.  gdata = (kappa, mu).
struct ModelImmigrationDeath {
    static constexpr int ID = M_IMMIGRATION_DEATH, NC = 1, NT = 2, NV = 0, NLD = 0, NGD = 2;
    static constexpr bool COUPLED = false, GENERATED = false;
    template <int J>
    __device__ static __forceinline__ double rate(const int32_t* u, const double*, const double*,
                                                  const double* gd) {
        if constexpr (J == 0)
            return gd[0];
        else
            return gd[1] * (double)u[0];
    }
    __device__ static __forceinline__ bool pts(double*, const int32_t*, const double*, const double*,
                                               int64_t) {
        return true;
    }
    // the post-time step leaves every state unchanged
    __device__ static __forceinline__ bool pts_fixed(const double*, const int32_t*) { return true; }
};

// Host-side table of model shapes.
struct ModelShape {
    int nc, nt, nv, nld, ngd;
};
inline bool model_shape(int id, ModelShape* s) {
    switch (id) {
        case M_SIR: *s = {3, 2, 0, 0, 2}; return true;
        case M_SIS: *s = {2, 2, 0, 0, 2}; return true;
        case M_SISE: *s = {2, 2, 1, 4, 7}; return true;
        case M_BIRTH_DEATH: *s = {1, 2, 0, 0, 2}; return true;
        case M_IMMIGRATION_DEATH: *s = {1, 2, 0, 0, 2}; return true;
        case M_SISE_SP: *s = {2, 2, 1, 4, 8}; return true;
    }
    return false;
}

}  // namespace siminf
