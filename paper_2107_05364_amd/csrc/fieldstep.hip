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
    const int s = blockIdx.y;
    const int a0 = blockIdx.x * TT;
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
    __shared__ float red[NW][TT * 3];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int t = 0; t < TT; ++t)
#pragma unroll
            for (int c = 0; c < 3; ++c) red[wave][3 * t + c] = acc[t][c];
    }
    __syncthreads();
    if (wave != 0) return;
    double rmax = 0.0, dmax = 0.0;
    if (lane < TT && a0 + lane < M.n) {
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
        if (lane == 0) {
            atomicMax(E.err + s, static_cast<unsigned long long>(__double_as_longlong(rmax)));
            atomicMax(E.dmx + s, static_cast<unsigned long long>(__double_as_longlong(dmax)));
        }
    }
}

template <int BLOCK, int TT, int NT, int WPE>
tm_status launch_tt(const DevProblem& P, const MvArgs& M, Epi mode, int64_t B, const EpiArgs& e,
                    hipStream_t st) {
    const dim3 grid(static_cast<unsigned>((M.n + TT - 1) / TT), static_cast<unsigned>(B));
    const dim3 block(BLOCK);
    switch (mode) {
        case Epi::HD: k_field<BLOCK, TT, NT, WPE, Epi::HD><<<grid, block, 0, st>>>(P, M, e); break;
        case Epi::HEFF: k_field<BLOCK, TT, NT, WPE, Epi::HEFF><<<grid, block, 0, st>>>(P, M, e); break;
        case Epi::DMDT: k_field<BLOCK, TT, NT, WPE, Epi::DMDT><<<grid, block, 0, st>>>(P, M, e); break;
        case Epi::STAGE: k_field<BLOCK, TT, NT, WPE, Epi::STAGE><<<grid, block, 0, st>>>(P, M, e); break;
        case Epi::RK4_FINAL:
            k_field<BLOCK, TT, NT, WPE, Epi::RK4_FINAL><<<grid, block, 0, st>>>(P, M, e);
            break;
        case Epi::DP_LAST:
            k_field<BLOCK, TT, NT, WPE, Epi::DP_LAST><<<grid, block, 0, st>>>(P, M, e);
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

// Per-state step control after the last stage (one thread per state).
__global__ void k_control(int64_t B, int integ, const double* __restrict__ prm,
                          double* __restrict__ t, double* __restrict__ h, double* __restrict__ dt,
                          unsigned long long* __restrict__ err, unsigned long long* __restrict__ dmx,
                          int64_t* __restrict__ steps, int64_t* __restrict__ rejected,
                          int32_t* __restrict__ flags, int32_t* __restrict__ acc) {
    const int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s >= B) return;
    const double t_end = prm[RP_TEND];
    const double max_steps = prm[RP_MAX_STEPS];
    const double e = __longlong_as_double(static_cast<long long>(err[s]));
    const double dm = __longlong_as_double(static_cast<long long>(dmx[s]));
    err[s] = 0ull;
    dmx[s] = 0ull;
    int32_t f = flags[s];
    if (f & (FLAG_DONE | FLAG_NONFINITE | FLAG_STEP)) {
        acc[s] = 0;
        h[s] = 0.0;
        return;
    }
    const double hh = h[s];
    double tn = t[s];
    bool done = false;
    if (integ == TM_RK4) {
        tn += hh;
        steps[s] += 1;
        acc[s] = 1;
        done = static_cast<double>(steps[s]) >= max_steps || (t_end > 0.0 && tn >= t_end);
        t[s] = tn;
        if (done) f |= FLAG_DONE;
        flags[s] = f;
        const double dn = dt[s];
        h[s] = done ? 0.0 : (t_end > 0.0 ? fmin(dn, t_end - tn) : dn);
        return;
    }
    if (!(e == e) || e == INFINITY || !(dm == dm)) {
        flags[s] = f | FLAG_NONFINITE;
        acc[s] = 0;
        h[s] = 0.0;
        return;
    }
    const bool ok = e <= 1.0;
    if (ok) {
        tn += hh;
        steps[s] += 1;
    } else {
        rejected[s] += 1;
    }
    acc[s] = ok ? 1 : 0;
    const double fac = (e == 0.0) ? 5.0 : fmin(5.0, fmax(0.2, 0.9 * pow(e, -0.2)));
    double dn = hh * fac;
    t[s] = tn;
    const bool converged = ok && prm[RP_DMDT_STOP] > 0.0 && dm < prm[RP_DMDT_STOP];
    done = static_cast<double>(steps[s]) >= max_steps || (t_end > 0.0 && tn >= t_end) || converged;
    // a state waiting for equilibrium that stops at the step cap is marked
    if (done && !converged && prm[RP_DMDT_STOP] > 0.0) f |= FLAG_CAPPED;
    if (t_end > 0.0 && tn + dn > t_end) dn = t_end - tn;
    dt[s] = done ? hh * fac : dn;
    if (done) {
        f |= FLAG_DONE;
    } else if (dn < prm[RP_DTMIN]) {
        f |= FLAG_STEP;
    }
    flags[s] = f;
    h[s] = (f & (FLAG_DONE | FLAG_STEP)) ? 0.0 : dn;
}

// Accept / reject (DP45): on acceptance y <- y5 (renormalised), k1 <- k7;
// then the next attempt's stage-2 input y + h a21 k1.
__global__ void k_commit(int32_t n, int64_t np, int64_t B, float* __restrict__ y,
                         float* __restrict__ k1, const float* __restrict__ y5,
                         const float* __restrict__ k7, float* __restrict__ ya,
                         const double* __restrict__ h, const int32_t* __restrict__ acc,
                         const double* __restrict__ prm) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= B * np) return;
    const int64_t s = i / np, a = i % np;
    if (a >= n) return;
    const int64_t o = s * 3 * np + 3 * a;
    float v0 = y[o], v1 = y[o + 1], v2 = y[o + 2];
    float g0 = k1[o], g1 = k1[o + 1], g2 = k1[o + 2];
    if (acc[s]) {
        v0 = y5[o]; v1 = y5[o + 1]; v2 = y5[o + 2];
        if (prm[RP_RENORM] != 0.0) {
            const float r = 1.0f / sqrtf(v0 * v0 + v1 * v1 + v2 * v2);
            v0 *= r; v1 *= r; v2 *= r;
        }
        g0 = k7[o]; g1 = k7[o + 1]; g2 = k7[o + 2];
        y[o] = v0; y[o + 1] = v1; y[o + 2] = v2;
        k1[o] = g0; k1[o + 1] = g1; k1[o + 2] = g2;
    }
    const float hh = static_cast<float>(h[s]) * (1.0f / 5.0f);
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

}  // namespace

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
    TM_REQUIRE(T->layout == TM_LAYOUT_SYM6 && T->prec == TM_PREC_FP32, TM_EINVAL,
               "field evaluation needs an FP32 SYM6 operator or a DENSE9 FP32 / BF16X3 / "
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
        case 0: return launch_tt<64, 2, 0, 8>(P, M, mode, B, e, s);
        case 1: return launch_tt<128, 2, 0, 8>(P, M, mode, B, e, s);
        case 2: return launch_tt<128, 4, 0, 8>(P, M, mode, B, e, s);
        case 3: return launch_tt<256, 2, 0, 8>(P, M, mode, B, e, s);
        case 4: return launch_tt<256, 4, 0, 8>(P, M, mode, B, e, s);
        case 5: return launch_tt<256, 8, 0, 8>(P, M, mode, B, e, s);
        case 6: return launch_tt<512, 4, 0, 8>(P, M, mode, B, e, s);
        case 7: return launch_tt<512, 8, 0, 8>(P, M, mode, B, e, s);
        case 8: return launch_tt<256, 2, 1, 8>(P, M, mode, B, e, s);
        case 9: return launch_tt<256, 4, 1, 8>(P, M, mode, B, e, s);
        case 10: return launch_tt<128, 1, 0, 8>(P, M, mode, B, e, s);
        case 11: return launch_tt<256, 1, 0, 8>(P, M, mode, B, e, s);
        case 12: return launch_tt<256, 4, 0, 2>(P, M, mode, B, e, s);
        case 13: return launch_tt<256, 8, 0, 2>(P, M, mode, B, e, s);
        case 14: return launch_tt<128, 4, 0, 2>(P, M, mode, B, e, s);
        case 15: return launch_tt<512, 8, 0, 2>(P, M, mode, B, e, s);
        default: break;
    }
    set_error("unknown field-kernel shape %d", shape);
    return TM_EINVAL;
}

int default_shape(int64_t n) {
    // narrow workgroups for short rows so that every lane streams data
    const int64_t ld = round_up(n, 4);
    if (ld <= 256) return 0;
    if (ld <= 1024) return 1;
    if (n <= 4096) return 4;
    return 5;
}

tm_status launch_pack(const float* src, int64_t B, int64_t n, int64_t np, float* dst,
                      hipStream_t s) {
    const int64_t cnt = B * np * 3;
    k_pack<<<static_cast<unsigned>((cnt + 255) / 256), 256, 0, s>>>(src, n, np, B, dst);
    TM_TRY_HIP(hipGetLastError());
    return TM_OK;
}

tm_status launch_control(Workspace* w, int64_t B, int integ, hipStream_t s) {
    k_control<<<static_cast<unsigned>((B + 255) / 256), 256, 0, s>>>(
        B, integ, w->params, w->t, w->h, w->dt, w->err, w->dmx, w->steps, w->rejected, w->flags,
        w->acc);
    TM_TRY_HIP(hipGetLastError());
    return TM_OK;
}

tm_status launch_commit(const Problem* p, Workspace* w, int64_t B, hipStream_t s) {
    const int64_t cnt = B * p->np;
    k_commit<<<static_cast<unsigned>((cnt + 255) / 256), 256, 0, s>>>(
        static_cast<int32_t>(p->n), p->np, B, w->y, w->k[0], w->y5, w->k[6], w->ya, w->h, w->acc,
        w->params);
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
