// Demag product fused with the local effective-field terms, the
// Landau-Lifshitz right-hand side and the Runge-Kutta stage update, plus the
// per-state step control, the accept/commit pass and the energy reduction.
//
// One workgroup owns TT target tiles of one state.  It streams their rows of
// the stored operator (SYM6: six planes xx, xy, xz, yy, yz, zz, each row
// contiguous over source tiles) once from memory with 16-byte loads, 4 source
// tiles per lane per step; the source state is read in the same step and
// reused by the TT rows.  After a fixed-order wave + LDS reduction the
// workgroup holds H_d = -N (Ms m) of its tiles (paper Sec. 2.3, Sec. 3.1) and
// finishes them in the same launch:
//   exchange  : sum_b w_ab (m_b - m_a), w_ab = 2A S_ab/(mu0 Ms_a V_a d_ab), a
//               missing neighbour contributes nothing (Neumann, Sec. 2.1);
//   anisotropy: (2K/(mu0 Ms)) (m . e) e;   applied field H_a  (Sec. 2.3);
//   LL        : dm/dt = -c1 m x H - c2 m x (m x H)             (Sec. 2.1);
//   stage     : next stage input y + h sum_j a_j k_j, or the RK4 update, or
//               the Dormand-Prince error estimate in float64 (Sec. 3.1).
// The reduction order depends only on the tile count, never on the batch,
// so a state's result does not depend on what it is batched with.
#include <cmath>

#include "common.h"
#include "epilogue.h"

namespace tmag {
namespace {

struct MvArgs {
    int32_t n;
    int64_t ld;     // SYM6 row stride (multiple of 4) = number of streamed columns
    int64_t plane;  // SYM6 plane stride
    const float* T;
    const float* Ms;  // [np]
    const float* X;   // [B][np][3]
    int64_t sx;       // 3 * np
};

typedef float f4v __attribute__((ext_vector_type(4)));

__device__ inline float4 ld4(const float* p) { return *reinterpret_cast<const float4*>(p); }

// Operator stream: each entry is read exactly once per launch, so NT = 1
// marks the loads nontemporal (the cache may drop the lines first).
template <int NT>
__device__ inline float4 ldT(const float* p) {
    if constexpr (NT) {
        const f4v v = __builtin_nontemporal_load(reinterpret_cast<const f4v*>(p));
        return make_float4(v.x, v.y, v.z, v.w);
    } else {
        return *reinterpret_cast<const float4*>(p);
    }
}

// WPE caps the waves per SIMD the compiler schedules for: with few resident
// waves a lower cap lets every 16-byte operator load of an iteration stay in
// flight at once (more registers per lane) instead of trading it for occupancy.
template <int BLOCK, int TT, int NT, int WPE, Epi MODE>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(1, WPE))) void k_field(
    DevProblem P, MvArgs M, EpiArgs E) {
    constexpr int NW = BLOCK / 64;
    constexpr bool STEPPING = MODE == Epi::STAGE || MODE == Epi::RK4_FINAL || MODE == Epi::DP_LAST;
    const int s = blockIdx.y;
    const int a0 = blockIdx.x * TT;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    rk4_last_stage_control<MODE>(E);
    // a state that is done or failed has h = 0: its stages are skipped (the
    // last stage still reports to the step control)
    bool frozen = false;
    if constexpr (STEPPING) frozen = E.h[s] == 0.0;
    if constexpr (MODE == Epi::STAGE || MODE == Epi::RK4_FINAL) {
        if (frozen) return;
    }
    __shared__ float red[NW][TT * 3];
    if (!frozen) {
        const float* x = M.X + s * M.sx;
        float acc[TT][3];
#pragma unroll
        for (int t = 0; t < TT; ++t) acc[t][0] = acc[t][1] = acc[t][2] = 0.0f;
        int64_t rowoff[TT];
#pragma unroll
        for (int t = 0; t < TT; ++t) rowoff[t] = static_cast<int64_t>(min(a0 + t, M.n - 1)) * M.ld;

        for (int64_t b = 4 * static_cast<int64_t>(threadIdx.x); b < M.ld; b += 4 * BLOCK) {
            const float4 q0 = ld4(x + 3 * b), q1 = ld4(x + 3 * b + 4), q2 = ld4(x + 3 * b + 8);
            const float4 ms = ld4(M.Ms + b);
            const float mx0 = q0.x * ms.x, mx1 = q0.w * ms.y, mx2 = q1.z * ms.z, mx3 = q2.y * ms.w;
            const float my0 = q0.y * ms.x, my1 = q1.x * ms.y, my2 = q1.w * ms.z, my3 = q2.z * ms.w;
            const float mz0 = q0.z * ms.x, mz1 = q1.y * ms.y, mz2 = q2.x * ms.z, mz3 = q2.w * ms.w;
#pragma unroll
            for (int t = 0; t < TT; ++t) {
                const float* tp = M.T + rowoff[t] + b;
                const float4 xx = ldT<NT>(tp), xy = ldT<NT>(tp + M.plane),
                             xz = ldT<NT>(tp + 2 * M.plane);
                const float4 yy = ldT<NT>(tp + 3 * M.plane), yz = ldT<NT>(tp + 4 * M.plane),
                             zz = ldT<NT>(tp + 5 * M.plane);
                float hx = acc[t][0], hy = acc[t][1], hz = acc[t][2];
                hx += xx.x * mx0 + xy.x * my0 + xz.x * mz0;
                hy += xy.x * mx0 + yy.x * my0 + yz.x * mz0;
                hz += xz.x * mx0 + yz.x * my0 + zz.x * mz0;
                hx += xx.y * mx1 + xy.y * my1 + xz.y * mz1;
                hy += xy.y * mx1 + yy.y * my1 + yz.y * mz1;
                hz += xz.y * mx1 + yz.y * my1 + zz.y * mz1;
                hx += xx.z * mx2 + xy.z * my2 + xz.z * mz2;
                hy += xy.z * mx2 + yy.z * my2 + yz.z * mz2;
                hz += xz.z * mx2 + yz.z * my2 + zz.z * mz2;
                hx += xx.w * mx3 + xy.w * my3 + xz.w * mz3;
                hy += xy.w * mx3 + yy.w * my3 + yz.w * mz3;
                hz += xz.w * mx3 + yz.w * my3 + zz.w * mz3;
                acc[t][0] = hx; acc[t][1] = hy; acc[t][2] = hz;
            }
        }
        // fixed-order reduction: butterfly inside each wave, then across waves
#pragma unroll
        for (int t = 0; t < TT; ++t)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                float v = acc[t][c];
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
                acc[t][c] = v;
            }
        if (lane == 0) {
#pragma unroll
            for (int t = 0; t < TT; ++t)
#pragma unroll
                for (int c = 0; c < 3; ++c) red[wave][3 * t + c] = acc[t][c];
        }
        __syncthreads();
    }
    if (wave != 0) return;
    double rmax = 0.0, dmax = 0.0;
    if (!frozen && lane < TT && a0 + lane < M.n) {
        float h[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float v = 0.0f;
#pragma unroll
            for (int w = 0; w < NW; ++w) v += red[w][3 * lane + c];
            h[c] = -v;
        }
        finish_tile<MODE>(P, M.X, M.sx, E, s, a0 + lane, h[0], h[1], h[2], &rmax, &dmax);
    }
    if constexpr (MODE == Epi::DP_LAST) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            rmax = fmax(rmax, __shfl_xor(rmax, off, 64));
            dmax = fmax(dmax, __shfl_xor(dmax, off, 64));
        }
        report_partials(E, rmax, dmax, lane);
    }
}

template <int BLOCK, int TT, int NT, int WPE>
tm_status launch_tt(const DevProblem& P, const MvArgs& M, Epi mode, int64_t B, const EpiArgs& e,
                    hipStream_t st) {
    const dim3 grid(static_cast<unsigned>((M.n + TT - 1) / TT), static_cast<unsigned>(B));
    const dim3 block(BLOCK);
    switch (mode) {
        case Epi::HD: launch_op(k_field<BLOCK, TT, NT, WPE, Epi::HD>, grid, block, st, P, M, e); break;
        case Epi::HEFF: launch_op(k_field<BLOCK, TT, NT, WPE, Epi::HEFF>, grid, block, st, P, M, e); break;
        case Epi::DMDT: launch_op(k_field<BLOCK, TT, NT, WPE, Epi::DMDT>, grid, block, st, P, M, e); break;
        case Epi::STAGE: launch_op(k_field<BLOCK, TT, NT, WPE, Epi::STAGE>, grid, block, st, P, M, e); break;
        case Epi::RK4_FINAL:
            launch_op(k_field<BLOCK, TT, NT, WPE, Epi::RK4_FINAL>, grid, block, st, P, M, e);
            break;
        case Epi::DP_LAST:
            launch_op(k_field<BLOCK, TT, NT, WPE, Epi::DP_LAST>, grid, block, st, P, M, e);
            break;
    }
    TM_TRY_HIP(hipGetLastError());
    return TM_OK;
}

// ---------------------------------------------------------------- elementwise

__global__ void k_pack(const float* __restrict__ src, int64_t n, int64_t np, int64_t B,
                       float* __restrict__ dst) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= B * np * 3) return;
    const int64_t s = i / (3 * np), r = i % (3 * np);
    dst[i] = (r < 3 * n) ? src[s * 3 * n + r] : 0.0f;
}

// RK4 step bookkeeping after the final stage (one thread per state).
__global__ void k_control_rk4(int64_t B, const double* __restrict__ prm, double* __restrict__ t,
                              double* __restrict__ h, double* __restrict__ dt,
                              int64_t* __restrict__ steps, int32_t* __restrict__ flags) {
    const int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s >= B) return;
    rk4_control(prm, t, h, dt, steps, flags, t, h, steps, flags, s);
}

// Accept / reject of a Dormand-Prince attempt.  Block (x, s) takes tiles
// [x kCommitTiles, (x + 1) kCommitTiles) of state s: it reduces the state's
// per-block error and |dm/dt| partials of the last stage, decides
// (dp_decide) from the control values the last stage copied (all blocks of a
// state decide alike; block 0 writes the new control values), and applies
// the step to its tiles -- on acceptance y <- y5 (renormalised), k1 <- k7 --
// then forms the next attempt's stage-2 input y + h a21 k1.  No block
// depends on another.
constexpr int kCommitThreads = 256;
constexpr int kCommitTiles = kCommitThreads;  // one tile per thread

__global__ __launch_bounds__(kCommitThreads) void k_commit(
    int32_t n, int64_t np, float* __restrict__ y, float* __restrict__ k1,
    const float* __restrict__ y5, const float* __restrict__ k7, float* __restrict__ ya,
    const double* __restrict__ errp, const double* __restrict__ dmxp, int64_t pstride, int64_t nblk,
    const double* __restrict__ snap, double* __restrict__ t, double* __restrict__ h,
    double* __restrict__ dt, int64_t* __restrict__ steps, int64_t* __restrict__ rejected,
    int32_t* __restrict__ flags, int32_t* __restrict__ acc, const double* __restrict__ prm) {
    constexpr int NW = kCommitThreads / 64;
    __shared__ double r0[NW], r1[NW];
    const int64_t s = blockIdx.y;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // everything the decision does not change is loaded first, so that its
    // latency overlaps the reduction: the control values and the tile's
    // candidate states and slopes
    const double* c = snap + s * kSnapStride;
    const double h0 = c[SN_H], t0 = c[SN_T], dt0 = c[SN_DT];
    const int64_t st0 = __double_as_longlong(c[SN_STEPS]), rj0 = __double_as_longlong(c[SN_REJ]);
    const int32_t f0 = static_cast<int32_t>(__double_as_longlong(c[SN_FLAGS]));
    const int64_t a = static_cast<int64_t>(blockIdx.x) * kCommitTiles + threadIdx.x;
    const bool mine = a < n;
    const int64_t o = s * 3 * np + 3 * a;
    float vy[3] = {}, vy5[3] = {}, vk1[3] = {}, vk7[3] = {};
    if (mine) {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            vy[q] = y[o + q];
            vy5[q] = y5[o + q];
            vk1[q] = k1[o + q];
            vk7[q] = k7[o + q];
        }
    }
    double e = 0.0, dm = 0.0;
    for (int64_t i = threadIdx.x; i < nblk; i += kCommitThreads) {
        e = fmax(e, errp[s * pstride + i]);
        dm = fmax(dm, dmxp[s * pstride + i]);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        e = fmax(e, __shfl_xor(e, off, 64));
        dm = fmax(dm, __shfl_xor(dm, off, 64));
    }
    if (lane == 0) {
        r0[wave] = e;
        r1[wave] = dm;
    }
    __syncthreads();
    e = r0[0];
    dm = r1[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) {
        e = fmax(e, r0[w]);
        dm = fmax(dm, r1[w]);
    }
    const Decision d = dp_decide(prm, e, dm, h0, t0, dt0, st0, rj0, f0);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        t[s] = d.t;
        dt[s] = d.dt;
        h[s] = d.h;
        steps[s] = d.steps;
        rejected[s] = d.rejected;
        flags[s] = d.flags;
        acc[s] = d.acc;
    }
    if (!mine) return;
    const bool renorm = prm[RP_RENORM] != 0.0;
    const float hh = static_cast<float>(d.h) * (1.0f / 5.0f);
    float v0, v1, v2, g0, g1, g2;
    if (d.acc) {
        v0 = vy5[0]; v1 = vy5[1]; v2 = vy5[2];
        if (renorm) {
            const float r = 1.0f / sqrtf(v0 * v0 + v1 * v1 + v2 * v2);
            v0 *= r; v1 *= r; v2 *= r;
        }
        g0 = vk7[0]; g1 = vk7[1]; g2 = vk7[2];
        y[o] = v0; y[o + 1] = v1; y[o + 2] = v2;
        k1[o] = g0; k1[o + 1] = g1; k1[o + 2] = g2;
    } else {
        v0 = vy[0]; v1 = vy[1]; v2 = vy[2];
        g0 = vk1[0]; g1 = vk1[1]; g2 = vk1[2];
    }
    ya[o] = v0 + hh * g0;
    ya[o + 1] = v1 + hh * g1;
    ya[o + 2] = v2 + hh * g2;
}

// Energy terms per state in float64: block partial sums, then a fixed-order
// final pass (paper Sec. 2.2-2.3 energy densities, integrated tile-wise).
__global__ __launch_bounds__(256) void k_energy_part(int32_t n, int64_t np, const float* __restrict__ X,
                                                     const float* __restrict__ Ha,
                                                     const float* __restrict__ Hd,
                                                     const double* __restrict__ vms,
                                                     const double* __restrict__ vk,
                                                     const float* __restrict__ easy,
                                                     const int32_t* __restrict__ nptr,
                                                     const int32_t* __restrict__ nidx,
                                                     const double* __restrict__ xw,
                                                     double* __restrict__ part) {
    const int s = blockIdx.y;
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    double ed = 0.0, ex = 0.0, ea = 0.0, ez = 0.0;
    if (a < n) {
        const float* x = X + static_cast<int64_t>(s) * 3 * np;
        const double m0 = x[3 * a], m1 = x[3 * a + 1], m2 = x[3 * a + 2];
        const float* hd = Hd + static_cast<int64_t>(s) * 3 * np + 3 * a;
        ed = -0.5 * kMu0 * vms[a] * (m0 * hd[0] + m1 * hd[1] + m2 * hd[2]);
        if (Ha) ez = -kMu0 * vms[a] * (m0 * Ha[3 * s] + m1 * Ha[3 * s + 1] + m2 * Ha[3 * s + 2]);
        if (easy) {
            const double me = m0 * easy[3 * a] + m1 * easy[3 * a + 1] + m2 * easy[3 * a + 2];
            ea = -vk[a] * me * me;
        }
        for (int32_t j = nptr[a]; j < nptr[a + 1]; ++j) {
            const int32_t b = nidx[j];
            if (b < a) continue;  // each face once
            const double d0 = x[3 * b] - m0, d1 = x[3 * b + 1] - m1, d2 = x[3 * b + 2] - m2;
            ex += xw[j] * (d0 * d0 + d1 * d1 + d2 * d2);
        }
    }
    __shared__ double red[4][256];
    red[0][threadIdx.x] = ed; red[1][threadIdx.x] = ex;
    red[2][threadIdx.x] = ea; red[3][threadIdx.x] = ez;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st)
            for (int c = 0; c < 4; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x < 4) part[(static_cast<int64_t>(s) * gridDim.x + blockIdx.x) * 4 + threadIdx.x] =
        red[threadIdx.x][0];
}

__global__ void k_energy_final(int64_t B, int64_t nblk, const double* __restrict__ part,
                               double* __restrict__ E) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= B * 4) return;
    const int64_t s = i / 4, c = i % 4;
    double v = 0.0;
    for (int64_t b = 0; b < nblk; ++b) v += part[(s * nblk + b) * 4 + c];
    E[i] = v;
}

// Diagnostics partials per block of 256 tiles and state, in float64:
// sum V Ms m (3), sum V Ms, max |dm/dt|, count of non-finite values.
__global__ __launch_bounds__(256) void k_diag_part(int32_t n, int64_t np, const float* __restrict__ X,
                                                   const float* __restrict__ Hd, const float* __restrict__ K,
                                                   const double* __restrict__ vms, double* __restrict__ part) {
    const int s = blockIdx.y;
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    double v[6] = {0, 0, 0, 0, 0, 0};
    if (a < n) {
        const int64_t o = static_cast<int64_t>(s) * 3 * np + 3 * a;
        const double w = vms[a];
        bool ok = true;
        double k2 = 0.0;
        for (int c = 0; c < 3; ++c) {
            const float m = X[o + c], h = Hd[o + c], k = K[o + c];
            ok = ok && isfinite(m) && isfinite(h) && isfinite(k);
            v[c] = w * m;
            k2 += static_cast<double>(k) * k;
        }
        v[3] = w;
        v[4] = ok ? sqrt(k2) : 0.0;
        v[5] = ok ? 0.0 : 1.0;
    }
    __shared__ double red[6][256];
    for (int c = 0; c < 6; ++c) red[c][threadIdx.x] = v[c];
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
            for (int c = 0; c < 4; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + st];
            red[4][threadIdx.x] = fmax(red[4][threadIdx.x], red[4][threadIdx.x + st]);
            red[5][threadIdx.x] += red[5][threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x < 6) part[(static_cast<int64_t>(s) * gridDim.x + blockIdx.x) * 6 + threadIdx.x] =
        red[threadIdx.x][0];
}

__global__ void k_diag_final(int64_t B, int64_t nblk, const double* __restrict__ part,
                             const double* __restrict__ E4, double* __restrict__ D) {
    const int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s >= B) return;
    double m0 = 0, m1 = 0, m2 = 0, w = 0, dm = 0, bad = 0;
    for (int64_t b = 0; b < nblk; ++b) {
        const double* q = part + (s * nblk + b) * 6;
        m0 += q[0]; m1 += q[1]; m2 += q[2]; w += q[3];
        dm = fmax(dm, q[4]);
        bad += q[5];
    }
    double* d = D + s * 9;
    for (int c = 0; c < 4; ++c) d[c] = E4[s * 4 + c];
    d[4] = m0 / w;
    d[5] = m1 / w;
    d[6] = m2 / w;
    d[7] = dm;
    d[8] = bad > 0.0 ? 1.0 : 0.0;
}

}  // namespace

tm_status launch_diagnostics(const Problem* p, int64_t B, const float* X, const float* Hd,
                             const float* dmdt, const double* E4, double* D, hipStream_t s) {
    Workspace* w = p->ws.get();
    const int64_t nblk = (p->n + 255) / 256;
    TM_REQUIRE(w && w->diag && w->B >= B, TM_EINVAL, "diagnostics workspace missing");
    k_diag_part<<<dim3(static_cast<unsigned>(nblk), static_cast<unsigned>(B)), 256, 0, s>>>(
        static_cast<int32_t>(p->n), p->np, X, Hd, dmdt, p->e_w, w->diag);
    TM_TRY_HIP(hipGetLastError());
    k_diag_final<<<static_cast<unsigned>((B + 255) / 256), 256, 0, s>>>(B, nblk, w->diag, E4, D);
    TM_TRY_HIP(hipGetLastError());
    return TM_OK;
}

DevProblem Problem::dev() const {
    DevProblem d;
    d.n = static_cast<int32_t>(n);
    d.np = static_cast<int32_t>(np);
    d.Ms = Ms;
    d.nbr_ptr = nbr_ptr;
    d.nbr_idx = nbr_idx;
    d.nbr_w = nbr_w;
    d.ku = ku;
    d.easy = easy;
    d.c1 = static_cast<float>(c1);
    d.c2 = static_cast<float>(c2);
    return d;
}

tm_status launch_field(const Problem* p, Epi mode, int64_t B, const float* X, const EpiArgs& e,
                       hipStream_t s) {
    const Tensor* T = p->T;
    if (T->layout == TM_LAYOUT_DENSE9 && T->prec != TM_PREC_FP64)
        return launch_field_batched(p, mode, B, X, e, s);
    if (T->layout == TM_LAYOUT_BSR6) return launch_field_bsr(p, mode, B, X, e, s);
    if (is_psym(T->layout)) return launch_field_psym(p, mode, B, X, e, s);
    TM_REQUIRE(T->layout == TM_LAYOUT_SYM6 && T->prec == TM_PREC_FP32, TM_EINVAL,
               "field evaluation needs an FP32 SYM6, BSR6, PSYM6 or PSYM4 operator or a DENSE9 FP32 / BF16X3 / "
               "FP16X3 operator (FP64 operators are for verification)");
    MvArgs M;
    M.n = static_cast<int32_t>(p->n);
    M.ld = T->ld;
    M.plane = T->plane;
    M.T = static_cast<const float*>(T->data);
    M.Ms = p->Ms;
    M.X = X;
    M.sx = 3 * p->np;
    const DevProblem P = p->dev();
    const int shape = p->shape >= 0 ? p->shape : default_shape(p->n);
    switch (shape) {
#define TM_SHAPE(i, BL, TT, NT, WPE) \
    case i: return launch_tt<BL, TT, NT, WPE>(P, M, mode, B, e, s);
        TM_FIELD_SHAPES(TM_SHAPE)
#undef TM_SHAPE
        default: break;
    }
    set_error("unknown field-kernel shape %d", shape);
    return TM_EINVAL;
}

int default_shape(int64_t n) {
    // measured on MI355X: one target tile per workgroup while the operator
    // is cache-sized; nontemporal streaming once it is far larger than the
    // 256 MB Infinity Cache
    const int64_t ld = round_up(n, 4);
    if (ld <= 256) return 0;
    if (ld <= 1024) return 10;
    if (n <= 8192) return 11;
    return 8;
}

tm_status launch_pack(const float* src, int64_t B, int64_t n, int64_t np, float* dst,
                      hipStream_t s) {
    const int64_t cnt = B * np * 3;
    k_pack<<<static_cast<unsigned>((cnt + 255) / 256), 256, 0, s>>>(src, n, np, B, dst);
    TM_TRY_HIP(hipGetLastError());
    return TM_OK;
}

tm_status launch_control(Workspace* w, int64_t B, int integ, hipStream_t s) {
    (void)integ;
    k_control_rk4<<<static_cast<unsigned>((B + 255) / 256), 256, 0, s>>>(B, w->params, w->t, w->h,
                                                                         w->dt, w->steps, w->flags);
    TM_TRY_HIP(hipGetLastError());
    return TM_OK;
}


int64_t last_stage_blocks(const Problem* p) {
    if (p->T->layout == TM_LAYOUT_DENSE9 && p->T->prec != TM_PREC_FP64) return (p->n + 255) / 256;
    if (p->T->layout == TM_LAYOUT_BSR6) return p->n;
    if (is_psym(p->T->layout)) return p->T->nt;
    static const int tt_of_shape[kNumShapes] = {
#define TM_SHAPE(i, BL, TT, NT, WPE) TT,
        TM_FIELD_SHAPES(TM_SHAPE)
#undef TM_SHAPE
    };
    const int sh = p->shape >= 0 ? p->shape : default_shape(p->n);
    return (p->n + tt_of_shape[sh] - 1) / tt_of_shape[sh];
}

tm_status launch_commit(const Problem* p, Workspace* w, int64_t B, hipStream_t s) {
    const dim3 grid(static_cast<unsigned>((p->n + kCommitTiles - 1) / kCommitTiles),
                    static_cast<unsigned>(B));
    k_commit<<<grid, kCommitThreads, 0, s>>>(
        static_cast<int32_t>(p->n), p->np, w->y, w->k[0], w->y5, w->k[6], w->ya, w->errp, w->dmxp,
        w->pstride, last_stage_blocks(p), w->snap, w->t, w->h, w->dt, w->steps, w->rejected,
        w->flags, w->acc, w->params);
    TM_TRY_HIP(hipGetLastError());
    return TM_OK;
}

tm_status launch_energy(const Problem* p, int64_t B, const float* X, const float* Ha,
                        const float* Hd, double* E, hipStream_t s) {
    Workspace* w = p->ws.get();
    const int64_t nblk = (p->n + 255) / 256;
    TM_REQUIRE(w && w->esum && w->esum_blocks >= nblk * B, TM_EINVAL, "energy workspace missing");
    k_energy_part<<<dim3(static_cast<unsigned>(nblk), static_cast<unsigned>(B)), 256, 0, s>>>(
        static_cast<int32_t>(p->n), p->np, X, Ha, Hd, p->e_w, p->e_vk, p->ku ? p->easy : nullptr,
        p->nbr_ptr, p->nbr_idx, p->x_w, w->esum);
    TM_TRY_HIP(hipGetLastError());
    k_energy_final<<<static_cast<unsigned>((B * 4 + 255) / 256), 256, 0, s>>>(B, nblk, w->esum, E);
    TM_TRY_HIP(hipGetLastError());
    return TM_OK;
}

}  // namespace tmag
