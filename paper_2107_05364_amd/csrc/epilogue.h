// Per-tile completion of a right-hand-side evaluation, shared by the fused
// matvec kernel and the elementwise pass of the batched (GEMM) path.
//
// Given H_d of tile a in state s, adds the local effective-field terms
// (paper Sec. 2.3: exchange sum_b w_ab (m_b - m_a) with w_ab = 2A S_ab /
// (mu0 Ms_a V_a d_ab) and zero flux through free faces; uniaxial anisotropy
// (2K/(mu0 Ms)) (m.e) e; applied field), evaluates the Landau-Lifshitz
// right-hand side -c1 m x H - c2 m x (m x H) (Sec. 2.1) and completes the
// requested Runge-Kutta stage (Sec. 3.1).
#pragma once

#include "common.h"

namespace tmag {
namespace {

// Dormand-Prince 5(4): fifth-order weights b and embedded fourth-order b*;
// the error weights are b - b*.
__device__ constexpr double kDpB[7] = {35.0 / 384, 0.0, 500.0 / 1113, 125.0 / 192,
                                       -2187.0 / 6784, 11.0 / 84, 0.0};
__device__ constexpr double kDpBs[7] = {5179.0 / 57600, 0.0, 7571.0 / 16695, 393.0 / 640,
                                        -92097.0 / 339200, 187.0 / 2100, 1.0 / 40};

// Local effective-field terms of tile a in state s (exchange, anisotropy,
// applied field), added to H; x is the state's stage input.
__device__ inline void add_local_field(const DevProblem& P, const float* __restrict__ x,
                                       const float* __restrict__ Ha, int s, int a, float m0, float m1,
                                       float m2, float& H0, float& H1, float& H2) {
    const int32_t j0 = P.nbr_ptr[a], j1 = P.nbr_ptr[a + 1];
    for (int32_t j = j0; j < j1; ++j) {
        const int32_t b = P.nbr_idx[j];
        const float w = P.nbr_w[j];
        H0 += w * (x[3 * b] - m0);
        H1 += w * (x[3 * b + 1] - m1);
        H2 += w * (x[3 * b + 2] - m2);
    }
    if (P.ku) {
        const float e0 = P.easy[3 * a], e1 = P.easy[3 * a + 1], e2 = P.easy[3 * a + 2];
        const float g = P.ku[a] * (m0 * e0 + m1 * e1 + m2 * e2);
        H0 += g * e0; H1 += g * e1; H2 += g * e2;
    }
    if (Ha) {
        H0 += Ha[3 * s]; H1 += Ha[3 * s + 1]; H2 += Ha[3 * s + 2];
    }
}

// Inputs of the epilogue that do not depend on the field: the tile's state
// m and, for the stepping modes, the previous stage slopes and the step's
// base state.  Loading them first lets a caller overlap their latency with
// the field's own reduction.
struct EpiIn {
    float m[3];
    float y[3];
    float kp[6][3];
};

template <Epi MODE>
__device__ inline void epi_load(const float* __restrict__ X, int64_t sx, const EpiArgs& E, int s, int a,
                                EpiIn& in) {
    const int64_t o = s * sx + 3 * static_cast<int64_t>(a);
    if constexpr (MODE != Epi::HD) {
#pragma unroll
        for (int c = 0; c < 3; ++c) in.m[c] = X[o + c];
    }
    if constexpr (MODE == Epi::STAGE || MODE == Epi::RK4_FINAL || MODE == Epi::DP_LAST) {
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            if (MODE == Epi::DP_LAST || j < E.nprev) {
#pragma unroll
                for (int c = 0; c < 3; ++c) in.kp[j][c] = E.kprev[j][o + c];
            }
        }
        const float* y = MODE == Epi::RK4_FINAL ? E.y_mut : E.y;
#pragma unroll
        for (int c = 0; c < 3; ++c) in.y[c] = y[o + c];
    }
}

// The epilogue proper from the whole effective field (H0, H1, H2) of tile a
// in state s: HD / HEFF store it, DMDT the Landau-Lifshitz right-hand side,
// the stepping modes complete their Runge-Kutta stage.
template <Epi MODE>
__device__ void epi_compute(const DevProblem& P, int64_t sx, const EpiArgs& E, int s, int a,
                            const EpiIn& in, float H0, float H1, float H2, double* rmax, double* dmax,
                            float* yn_out = nullptr) {
    const int64_t o = s * sx + 3 * static_cast<int64_t>(a);
    if constexpr (MODE == Epi::HD || MODE == Epi::HEFF) {
        float* out = E.out + s * E.out_stride + 3 * static_cast<int64_t>(a);
        out[0] = H0; out[1] = H1; out[2] = H2;
        return;
    } else {
        const float m0 = in.m[0], m1 = in.m[1], m2 = in.m[2];
        // m x H and m x (m x H)
        const float p0 = m1 * H2 - m2 * H1, p1 = m2 * H0 - m0 * H2, p2 = m0 * H1 - m1 * H0;
        const float q0 = m1 * p2 - m2 * p1, q1 = m2 * p0 - m0 * p2, q2 = m0 * p1 - m1 * p0;
        const float k0 = -P.c1 * p0 - P.c2 * q0;
        const float k1 = -P.c1 * p1 - P.c2 * q1;
        const float k2 = -P.c1 * p2 - P.c2 * q2;
        if constexpr (MODE == Epi::DMDT) {
            float* out = E.out + s * E.out_stride + 3 * static_cast<int64_t>(a);
            out[0] = k0; out[1] = k1; out[2] = k2;
            return;
        } else if constexpr (MODE == Epi::STAGE) {
            float* out = E.out + o;
            out[0] = k0; out[1] = k1; out[2] = k2;
            const float h = static_cast<float>(E.h[s]);
            float c0 = E.coef[E.nprev] * k0, c1 = E.coef[E.nprev] * k1, c2 = E.coef[E.nprev] * k2;
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                if (j < E.nprev) {
                    c0 += E.coef[j] * in.kp[j][0]; c1 += E.coef[j] * in.kp[j][1]; c2 += E.coef[j] * in.kp[j][2];
                }
            }
            float* yn = E.ynext + o;
            yn[0] = in.y[0] + h * c0; yn[1] = in.y[1] + h * c1; yn[2] = in.y[2] + h * c2;
            if (yn_out) {  // the stored values, for a caller that converts them further
                yn_out[0] = yn[0]; yn_out[1] = yn[1]; yn_out[2] = yn[2];
            }
            return;
        } else if constexpr (MODE == Epi::RK4_FINAL) {
            const double hd = E.h[s];
            if (hd == 0.0) return;
            const float h = static_cast<float>(hd);
            float c0 = E.coef[E.nprev] * k0, c1 = E.coef[E.nprev] * k1, c2 = E.coef[E.nprev] * k2;
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                if (j < E.nprev) {
                    c0 += E.coef[j] * in.kp[j][0]; c1 += E.coef[j] * in.kp[j][1]; c2 += E.coef[j] * in.kp[j][2];
                }
            }
            float v0 = in.y[0] + h * c0, v1 = in.y[1] + h * c1, v2 = in.y[2] + h * c2;
            if (E.renorm) {
                const float r = 1.0f / sqrtf(v0 * v0 + v1 * v1 + v2 * v2);
                v0 *= r; v1 *= r; v2 *= r;
            }
            float* y = E.y_mut + o;
            y[0] = v0; y[1] = v1; y[2] = v2;
            return;
        } else {  // DP_LAST: k7 at the fifth-order solution, float64 error estimate
            float* out = E.out + o;
            out[0] = k0; out[1] = k1; out[2] = k2;
            const double h = E.h[s];
            double e0 = (kDpB[6] - kDpBs[6]) * k0, e1 = (kDpB[6] - kDpBs[6]) * k1,
                   e2 = (kDpB[6] - kDpBs[6]) * k2;
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                const double w = kDpB[j] - kDpBs[j];
                e0 += w * in.kp[j][0]; e1 += w * in.kp[j][1]; e2 += w * in.kp[j][2];
            }
            const double atol = E.params[RP_ATOL], rtol = E.params[RP_RTOL];
            const double s0 = atol + rtol * fmax(fabs((double)in.y[0]), fabs((double)m0));
            const double s1 = atol + rtol * fmax(fabs((double)in.y[1]), fabs((double)m1));
            const double s2 = atol + rtol * fmax(fabs((double)in.y[2]), fabs((double)m2));
            const double r0 = fabs(h * e0) / s0, r1 = fabs(h * e1) / s1, r2 = fabs(h * e2) / s2;
            // a NaN anywhere must win the max: map it to +inf (fmax drops NaN)
            const bool bad = !(r0 == r0) || !(r1 == r1) || !(r2 == r2);
            *rmax = bad ? INFINITY : fmax(r0, fmax(r1, r2));
            const double d = sqrt((double)k0 * k0 + (double)k1 * k1 + (double)k2 * k2);
            *dmax = (d == d) ? d : INFINITY;
            return;
        }
    }
}

// Whole epilogue from H_d of tile a in state s.  LOCAL = false: (hd0, hd1,
// hd2) already holds the whole effective field (the caller added the local
// terms).
template <Epi MODE, bool LOCAL = true>
__device__ void finish_tile(const DevProblem& P, const float* __restrict__ X, int64_t sx,
                            const EpiArgs& E, int s, int a, float hd0, float hd1, float hd2,
                            double* rmax, double* dmax, float* yn_out = nullptr) {
    EpiIn in;
    epi_load<MODE>(X, sx, E, s, a, in);
    float H0 = hd0, H1 = hd1, H2 = hd2;
    if constexpr (LOCAL && MODE != Epi::HD)
        add_local_field(P, X + s * sx, E.Ha, s, a, in.m[0], in.m[1], in.m[2], H0, H1, H2);
    epi_compute<MODE>(P, sx, E, s, a, in, H0, H1, H2, rmax, dmax, yn_out);
}


// RK4 step control of state s after its step of length h: t += h, one more
// step, done at the step cap or at t_end; the next step is min(dt, t_end -
// t), 0 when done or stopped.  Reads (t, h, steps, flags) and writes (to,
// ho, so, fo): the same arrays for the control pass, the second set when the
// last stage advances the control.
__device__ inline void rk4_control(const double* __restrict__ prm, const double* t, const double* h,
                                   const double* __restrict__ dt, const int64_t* steps, const int32_t* flags,
                                   double* to, double* ho, int64_t* so, int32_t* fo, int64_t s) {
    int32_t f = flags[s];
    const double t0 = t[s], h0 = h[s];
    const int64_t st0 = steps[s];
    if (f & (FLAG_DONE | FLAG_NONFINITE | FLAG_STEP)) {
        to[s] = t0;
        so[s] = st0;
        fo[s] = f;
        ho[s] = 0.0;
        return;
    }
    const double t_end = prm[RP_TEND];
    const double tn = t0 + h0;
    const int64_t sn = st0 + 1;
    const bool done = static_cast<double>(sn) >= prm[RP_MAX_STEPS] || (t_end > 0.0 && tn >= t_end);
    if (done) f |= FLAG_DONE;
    to[s] = tn;
    so[s] = sn;
    fo[s] = f;
    const double dn = dt[s];
    ho[s] = done ? 0.0 : (t_end > 0.0 ? fmin(dn, t_end - tn) : dn);
}

// The last RK4 stage's share of the control: the first workgroup of each
// state (before anything else, also for a frozen state) advances it.
template <Epi MODE>
__device__ inline void rk4_last_stage_control(const EpiArgs& E) {
    if constexpr (MODE == Epi::RK4_FINAL) {
        if (E.rk_t_out && blockIdx.x == 0 && threadIdx.x == 0)
            rk4_control(E.params, E.t, E.h, E.dt, E.steps, E.flags, E.rk_t_out, E.rk_h_out, E.rk_steps_out,
                        E.rk_flags_out, blockIdx.y);
    }
}

// Dormand-Prince step control of one state: acceptance from the scaled
// max-norm error e (accept iff e <= 1), next step h * min(5, max(0.2,
// 0.9 e^-1/5)) (5 when e == 0), capped at t_end; done at the step cap, at
// t_end, or (accepted) when max_a |dm/dt|_a falls below the threshold.
struct Decision {
    int acc;
    double t, dt, h;
    int64_t steps, rejected;
    int32_t flags;
};

__device__ Decision dp_decide(const double* __restrict__ prm, double e, double dm, double hh,
                              double t, double dt, int64_t steps, int64_t rej, int32_t f) {
    Decision d{0, t, dt, 0.0, steps, rej, f};
    if (f & (FLAG_DONE | FLAG_NONFINITE | FLAG_STEP)) return d;
    if (!(e == e) || e == INFINITY || !(dm == dm)) {
        d.flags = f | FLAG_NONFINITE;
        return d;
    }
    const double t_end = prm[RP_TEND];
    const bool ok = e <= 1.0;
    if (ok) {
        d.t = t + hh;
        d.steps = steps + 1;
    } else {
        d.rejected = rej + 1;
    }
    d.acc = ok ? 1 : 0;
    const double fac = (e == 0.0) ? 5.0 : fmin(5.0, fmax(0.2, 0.9 * pow(e, -0.2)));
    double dn = hh * fac;
    const bool converged = ok && prm[RP_DMDT_STOP] > 0.0 && dm < prm[RP_DMDT_STOP];
    const bool done = static_cast<double>(d.steps) >= prm[RP_MAX_STEPS] ||
                      (t_end > 0.0 && d.t >= t_end) || converged;
    if (done && !converged && prm[RP_DMDT_STOP] > 0.0) d.flags |= FLAG_CAPPED;
    if (t_end > 0.0 && d.t + dn > t_end) dn = t_end - d.t;
    d.dt = done ? hh * fac : dn;
    if (done)
        d.flags |= FLAG_DONE;
    else if (dn < prm[RP_DTMIN])
        d.flags |= FLAG_STEP;
    d.h = (d.flags & (FLAG_DONE | FLAG_STEP)) ? 0.0 : dn;
    return d;
}

// Last stage: store the block's maxima (already reduced over the wave) for
// the commit pass, which reduces them per state.  The first block of each
// state also copies the state's control values, so that every block of the
// commit decides from the same inputs while one of them rewrites them.
__device__ inline void report_partials(const EpiArgs& E, double rmax, double dmax, int lane) {
    if (lane == 0) {
        const int64_t s = blockIdx.y;
        E.errp[s * E.pstride + blockIdx.x] = rmax;
        E.dmxp[s * E.pstride + blockIdx.x] = dmax;
        if (blockIdx.x == 0) {
            double* c = E.snap + s * kSnapStride;
            c[SN_H] = E.h[s];
            c[SN_T] = E.t[s];
            c[SN_DT] = E.dt[s];
            c[SN_STEPS] = __longlong_as_double(static_cast<long long>(E.steps[s]));
            c[SN_REJ] = __longlong_as_double(static_cast<long long>(E.rejected[s]));
            c[SN_FLAGS] = __longlong_as_double(static_cast<long long>(E.flags[s]));
        }
    }
}

}  // namespace
}  // namespace tmag
