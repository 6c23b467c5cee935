// Persistent fused RK4 integration of one state whose operator fits on the
// chip (paper Sec. 3.1: the effective field, an affine function of m, is
// applied at every stage of the explicit Runge-Kutta step).
//
// For a small mesh (at most kPersistMaxTiles tiles) a step is four field
// evaluations of a few microseconds each, so separate launches spend most of
// the step in launch and ramp.  Here one cooperative launch runs every step:
//  * workgroup g owns TT consecutive target tiles; at the start it copies
//    their six operator rows ([6][TT][np], float32) into LDS, where they stay
//    for the whole run;
//  * per stage it copies the whole stage input from a double-buffered global
//    array into LDS (m and Ms m), forms the demag sums of its tiles from LDS
//    (lane j of row r takes sources j, j + L, ...; a fixed shuffle tree
//    reduces the L lanes), and the first TT lanes of wave 0 add the local
//    terms, evaluate the LL slope, advance their tiles' RK4 registers and
//    write their share of the next stage input;
//  * a grid barrier ends the stage: wave 0 releases its stores at agent
//    scope, thread 0 increments a counter and spins (bounded) until every
//    workgroup has arrived, then acquires.
// The step control (fixed dt, t_end, step cap) is replayed identically by
// every workgroup; workgroup 0 writes the final control values.
#include <hip/hip_runtime.h>

#include "common.h"
#include "epilogue.h"

namespace tmag {
namespace {

constexpr int kPersistThreads = 256;
constexpr int kSpinCap = 1 << 20;  // polls of the barrier counter (about a second) before a workgroup gives up

struct PersistArgs {
    DevProblem P;
    const float* T;       // SYM6 planes [6][n][ld]
    int64_t ld, plane;
    float* X0;            // stage input, double-buffered [2][np][3]
    float* X1;
    float* y;             // [np][3] state in / out
    const float* Ha;      // [3]
    double* t;            // control values of the state (in / out)
    double* h;
    const double* dt;
    int64_t* steps;
    int32_t* flags;
    const double* prm;    // run parameters
    unsigned* bar;        // barrier counter, zero at launch
    int32_t* fail;        // set when a barrier wait gave up
};

// Grid barrier number k (k >= 1): every workgroup adds one to the counter;
// the barrier is passed when it reaches k * gridDim.x.  Wave 0 made the
// workgroup's global stores; its agent-scope release fence makes them
// visible before the increment, thread 0's agent-scope acquire fence after
// the wait makes the other workgroups' stores visible to this workgroup.
__device__ inline void grid_barrier(unsigned* bar, unsigned k, int32_t* fail) {
    if (threadIdx.x < 64) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned target = k * gridDim.x;
        int spins = 0;
        while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (++spins > kSpinCap) {
                atomicExch(fail, 1);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}

template <int TT>
__global__ __launch_bounds__(kPersistThreads) void k_rk4_persistent(PersistArgs A) {
    constexpr int L = kPersistThreads / TT;  // lanes per target row
    extern __shared__ float lds[];
    const DevProblem& P = A.P;
    const int np = P.np, n = P.n;
    float* opl = lds;                        // [6][TT][np]
    float* xs = opl + 6 * TT * np;           // [np][3] stage input m
    float* xw = xs + 3 * np;                 // [np][3] Ms m
    __shared__ float hsum[TT][3];
    const int t = threadIdx.x, r = t / L, j = t % L;
    const int a0 = blockIdx.x * TT;
    for (int i = t; i < 6 * TT * np; i += kPersistThreads) {
        const int c = i / (TT * np), rr = (i / np) % TT, b = i % np;
        const int a = a0 + rr;
        opl[i] = (a < n && b < n) ? A.T[c * A.plane + static_cast<int64_t>(a) * A.ld + b] : 0.0f;
    }
    // RK4 registers of tile a0 + t (lanes t < TT of wave 0)
    const bool owner = t < TT && a0 + t < n;
    const int ao = a0 + t;
    float y[3] = {}, k1[3] = {}, k2[3] = {}, k3[3] = {};
    if (owner) {
        for (int c = 0; c < 3; ++c) {
            y[c] = A.y[3 * ao + c];
            A.X0[3 * ao + c] = y[c];
        }
    }
    double tt = *A.t, hh = *A.h;
    const double dtf = *A.dt;
    int64_t steps = *A.steps;
    int32_t flags = *A.flags;
    const double t_end = A.prm[RP_TEND], max_steps = A.prm[RP_MAX_STEPS];
    const bool renorm = A.prm[RP_RENORM] != 0.0;
    unsigned k = 1;
    grid_barrier(A.bar, k++, A.fail);
    const float kFin[4] = {static_cast<float>(1.0 / 6), static_cast<float>(2.0 / 6), static_cast<float>(2.0 / 6),
                           static_cast<float>(1.0 / 6)};
    unsigned g = 0;  // stage count: input buffer g & 1
    while (!(flags & FLAG_DONE)) {
        const float h = static_cast<float>(hh);
        for (int st = 0; st < 4; ++st, ++g) {
            const float* Xin = (g & 1) ? A.X1 : A.X0;
            float* Xout = (g & 1) ? A.X0 : A.X1;
            for (int i = t; i < 3 * np; i += kPersistThreads) {
                const float v = i < 3 * n ? Xin[i] : 0.0f;
                xs[i] = v;
                xw[i] = v * P.Ms[i / 3];
            }
            __syncthreads();
            float s0 = 0.f, s1 = 0.f, s2 = 0.f;
            const float* o = opl + r * np;
            for (int b = j; b < np; b += L) {
                const float w0 = xw[3 * b], w1 = xw[3 * b + 1], w2 = xw[3 * b + 2];
                const float v0 = o[b], v1 = o[TT * np + b], v2 = o[2 * TT * np + b];
                const float v3 = o[3 * TT * np + b], v4 = o[4 * TT * np + b], v5 = o[5 * TT * np + b];
                s0 += v0 * w0 + v1 * w1 + v2 * w2;
                s1 += v1 * w0 + v3 * w1 + v4 * w2;
                s2 += v2 * w0 + v4 * w1 + v5 * w2;
            }
#pragma unroll
            for (int off = L / 2; off > 0; off >>= 1) {
                s0 += __shfl_xor(s0, off, 64);
                s1 += __shfl_xor(s1, off, 64);
                s2 += __shfl_xor(s2, off, 64);
            }
            if (j == 0) {
                hsum[r][0] = s0;
                hsum[r][1] = s1;
                hsum[r][2] = s2;
            }
            __syncthreads();
            if (owner) {
                const float m0 = xs[3 * ao], m1 = xs[3 * ao + 1], m2 = xs[3 * ao + 2];
                float H0 = -hsum[t][0], H1 = -hsum[t][1], H2 = -hsum[t][2];
                add_local_field(P, xs, A.Ha, 0, ao, m0, m1, m2, H0, H1, H2);
                const float p0 = m1 * H2 - m2 * H1, p1 = m2 * H0 - m0 * H2, p2 = m0 * H1 - m1 * H0;
                const float q0 = m1 * p2 - m2 * p1, q1 = m2 * p0 - m0 * p2, q2 = m0 * p1 - m1 * p0;
                const float kk[3] = {-P.c1 * p0 - P.c2 * q0, -P.c1 * p1 - P.c2 * q1, -P.c1 * p2 - P.c2 * q2};
                float nx[3];
                if (st < 3) {
                    for (int c = 0; c < 3; ++c) {
                        if (st == 0) k1[c] = kk[c];
                        if (st == 1) k2[c] = kk[c];
                        if (st == 2) k3[c] = kk[c];
                        nx[c] = y[c] + h * ((st == 2 ? 1.0f : 0.5f) * kk[c]);
                    }
                } else {
                    for (int c = 0; c < 3; ++c) {
                        const float cc = kFin[3] * kk[c] + kFin[0] * k1[c] + kFin[1] * k2[c] + kFin[2] * k3[c];
                        nx[c] = y[c] + h * cc;
                    }
                    if (renorm) {
                        const float q = 1.0f / sqrtf(nx[0] * nx[0] + nx[1] * nx[1] + nx[2] * nx[2]);
                        nx[0] *= q;
                        nx[1] *= q;
                        nx[2] *= q;
                    }
                    for (int c = 0; c < 3; ++c) y[c] = nx[c];
                }
                for (int c = 0; c < 3; ++c) Xout[3 * ao + c] = nx[c];
            }
            grid_barrier(A.bar, k++, A.fail);
        }
        // step control, as the launch-per-stage path does it
        const double tn = tt + hh;
        steps += 1;
        tt = tn;
        const bool done = static_cast<double>(steps) >= max_steps || (t_end > 0.0 && tn >= t_end);
        if (done) flags |= FLAG_DONE;
        hh = done ? 0.0 : (t_end > 0.0 ? fmin(dtf, t_end - tn) : dtf);
        if (__hip_atomic_load(A.fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
    }
    if (owner)
        for (int c = 0; c < 3; ++c) A.y[3 * ao + c] = y[c];
    if (blockIdx.x == 0 && t == 0) {
        *A.t = tt;
        *A.h = hh;
        *A.steps = steps;
        *A.flags = flags;
    }
}

__global__ void k_zero_u32(unsigned* p, int32_t* q) {
    if (threadIdx.x == 0) {
        *p = 0u;
        *q = 0;
    }
}

template <int TT>
tm_status launch_persistent_t(const Problem* p, Workspace* w, const tm_run_cfg* cfg, hipStream_t s) {
    (void)cfg;
    const Tensor* T = p->T;
    const int64_t np = p->np;
    const size_t lds = static_cast<size_t>(6 * TT * np + 6 * np) * sizeof(float);
    const auto kern = k_rk4_persistent<TT>;
    TM_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                   static_cast<int>(lds)));
    int per_cu = 0, cus = 0, dev = 0;
    TM_TRY_HIP(hipGetDevice(&dev));
    TM_TRY_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    TM_TRY_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kern),
                                                             kPersistThreads, lds));
    const int64_t G = (p->n + TT - 1) / TT;
    TM_REQUIRE(per_cu >= 1 && G <= static_cast<int64_t>(per_cu) * cus, TM_EINVAL,
               "persistent RK4: %lld workgroups cannot be co-resident (%d per CU, %d CUs)",
               static_cast<long long>(G), per_cu, cus);
    k_zero_u32<<<1, 64, 0, s>>>(w->bar, w->bar_fail);
    TM_TRY_HIP(hipGetLastError());
    PersistArgs A;
    A.P = p->dev();
    A.T = static_cast<const float*>(T->data);
    A.ld = T->ld;
    A.plane = T->plane;
    A.X0 = w->ya;
    A.X1 = w->yb;
    A.y = w->y;
    A.Ha = w->Ha;
    A.t = w->t;
    A.h = w->h;
    A.dt = w->dt;
    A.steps = w->steps;
    A.flags = w->flags;
    A.prm = w->params;
    A.bar = w->bar;
    A.fail = w->bar_fail;
    void* args[] = {&A};
    TM_TRY_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kern), dim3(static_cast<unsigned>(G)),
                                          dim3(kPersistThreads), args, static_cast<unsigned>(lds), s));
    return TM_OK;
}

}  // namespace

bool persistent_eligible(const Problem* p, int integ, int64_t B) {
    return integ == TM_RK4 && B == 1 && p->T->layout == TM_LAYOUT_SYM6 && p->T->prec == TM_PREC_FP32 &&
           p->np <= kPersistMaxTiles;
}

tm_status launch_persistent_rk4(const Problem* p, Workspace* w, const tm_run_cfg* cfg, hipStream_t s) {
    TM_REQUIRE(w->bar && w->bar_fail, TM_EINVAL, "persistent RK4: workspace has no barrier counter");
    if (p->np <= 512) return launch_persistent_t<8>(p, w, cfg, s);
    return launch_persistent_t<4>(p, w, cfg, s);
}

}  // namespace tmag
