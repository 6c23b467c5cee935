// Batched demag product on the matrix cores: many states that share one
// geometry turn H_d = -N (Ms m) into one GEMM per right-hand-side evaluation
// (paper Sec. 3.1: the demag operator is a dense 3N x 3N matrix applied to
// the 3N-vector m; here to B such vectors at once).
//
//   C[r][s] = sum_k A[r][k] X[s][k],  A = stored operator (DENSE9, row-major,
//   K contiguous), X[s][3b+j] = (Ms_b / Ms_ref) m_{s,b,j}, H_d = -Ms_ref C.
//
// Precisions (accumulation always float32):
//   FP32   : v_mfma_f32_16x16x4_f32, A and X in float32;
//   BF16X3 : A = Ah + Al, X = Xh + Xl in bf16; C = Ah Xh + Ah Xl + Al Xh
//            with v_mfma_f32_16x16x32_bf16 (the lo*lo term is below the
//            float32 rounding of the result);
//   FP16X3 : as BF16X3 with fp16 and a power-of-two scale per operator row
//            (the row maximum maps to 2^13..2^14, far entries stay normal);
//            the scale is removed in the GEMM epilogue.
//
// Work split: a workgroup (4 waves) owns 128 operator rows x all states and
// one K range (split-K); each wave owns two 16-row MFMA tiles.  The X chunk
// of the K range is staged once per workgroup in LDS (row-padded so the
// 16-byte reads of 16 lanes hit distinct banks) and reused by the 8 row
// tiles; operator rows are read straight from memory, 16 bytes per lane,
// each 128-byte line fully used.  Partial sums go to part[split][state][row]
// and a fixed-order elementwise pass adds the splits, finishes the
// effective field and the Runge-Kutta stage per tile.  The summation order
// depends only on the problem size, never on the batch.
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include "common.h"
#include "epilogue.h"

namespace tmag {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));

constexpr int kRowsPerBlock = 128;  // 4 waves x 2 tiles x 16 rows
constexpr int kKC = 128;            // largest K chunk (X double-buffered in LDS); ld is a multiple

// K chunk per (precision, state tiles), measured on the film operator
// (7680 x 7680): the split forms at 128 states and FP32 at 32-64 states run
// faster with 64-element chunks (half the registers and LDS: two workgroups
// per CU), the rest with 128.
constexpr int chunk_for(int prec, int nst) {
    return (prec != 0 && nst == 8) || (prec == 0 && (nst == 2 || nst == 4)) ? 64 : 128;
}

struct GemmArgs {
    int64_t ld;         // K extent (= 3 np) and operator row stride
    int64_t bpad;       // padded state count (multiple of 16)
    const void* Ahi;    // FP32: the operator; split: hi part
    const void* Alo;    // split: lo part
    const float* rscale;// FP16X3: 1/scale per row
    const void* Xhi;    // [bpad][ld]
    const void* Xlo;
    float* part;        // [splits][bpad][rows]
    int64_t rows;       // padded operator rows (multiple of 128)
    int64_t kper;       // K elements per split (multiple of the chunk)
};

template <int PREC>
struct Elt;
template <>
struct Elt<0> { using T = float; static constexpr int kPerLane = 4; };
template <>
struct Elt<1> { using T = __bf16; static constexpr int kPerLane = 8; };
template <>
struct Elt<2> { using T = _Float16; static constexpr int kPerLane = 8; };

// LDS row of one state's chunk: KC elements + 16 bytes of padding
template <int PREC, int KC>
constexpr int lds_row_bytes() { return KC * static_cast<int>(sizeof(typename Elt<PREC>::T)) + 16; }

// Software pipeline per K chunk c (KC = 64 or 128): the operator rows and the X
// tile of chunk c+1 are loaded into registers while the MFMAs of chunk c run
// from LDS buffer c&1; the X tile then goes to buffer (c+1)&1, which no wave
// reads any more (all passed the barrier after chunk c-1).  One barrier per
// chunk.  A chunk carries enough MFMA work (split: 192 per wave) to cover
// the latency of the next chunk's loads, and MFMAs are issued across
// independent accumulators so that none waits for its predecessor.
template <int PREC, int NST, int KC>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs G) {
    using T = typename Elt<PREC>::T;
    constexpr bool SPLIT = PREC != 0;
    constexpr int RB = lds_row_bytes<PREC, KC>();
    constexpr int NS = NST * 16;
    constexpr int CHUNK16 = KC * static_cast<int>(sizeof(T)) / 16;  // 16-byte pieces per state row
    constexpr int XPIECES = NS * CHUNK16;
    constexpr int XPT = (XPIECES + 255) / 256;  // pieces per thread and array
    constexpr int BUF = NS * RB * (SPLIT ? 2 : 1);
    constexpr int NSUB = PREC == 0 ? KC / 16 : KC / 32;
    using AV = typename std::conditional<PREC == 0, float4,
                                         typename std::conditional<PREC == 1, v8bf, v8h>::type>::type;
    __shared__ __attribute__((aligned(16))) unsigned char lds[2 * BUF];

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = lane >> 4, j = lane & 15;
    const int64_t rowbase = static_cast<int64_t>(blockIdx.x) * kRowsPerBlock + wave * 32;
    const int64_t kb = static_cast<int64_t>(blockIdx.y) * G.kper;
    const int64_t ke = min(kb + G.kper, G.ld);
    const int nch = static_cast<int>((ke - kb) / KC);

    const T* Ah = static_cast<const T*>(G.Ahi);
    const T* Al = static_cast<const T*>(G.Alo);
    const unsigned char* Xh = static_cast<const unsigned char*>(G.Xhi);
    const unsigned char* Xl = static_cast<const unsigned char*>(G.Xlo);
    const int64_t xrow = G.ld * static_cast<int64_t>(sizeof(T));  // bytes per state row

    v4f acc[2][NST];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int s = 0; s < NST; ++s) acc[r][s] = v4f{0.f, 0.f, 0.f, 0.f};

    v4u xh_r[XPT], xl_r[XPT];
    AV ah_r[NSUB][2], al_r[NSUB][2], ah_n[NSUB][2], al_n[NSUB][2];

    auto load_x = [&](int64_t k0) {
#pragma unroll
        for (int q = 0; q < XPT; ++q) {
            const int idx = threadIdx.x + 256 * q;
            if (XPIECES % 256 == 0 || idx < XPIECES) {
                const int st = idx / CHUNK16, pc = idx % CHUNK16;
                const int64_t off = st * xrow + k0 * static_cast<int64_t>(sizeof(T)) + 16 * pc;
                xh_r[q] = *reinterpret_cast<const v4u*>(Xh + off);
                if constexpr (SPLIT) xl_r[q] = *reinterpret_cast<const v4u*>(Xl + off);
            }
        }
    };
    auto store_x = [&](int buf) {
        unsigned char* base = lds + buf * BUF;
#pragma unroll
        for (int q = 0; q < XPT; ++q) {
            const int idx = threadIdx.x + 256 * q;
            if (XPIECES % 256 == 0 || idx < XPIECES) {
                const int st = idx / CHUNK16, pc = idx % CHUNK16;
                *reinterpret_cast<v4u*>(base + st * RB + 16 * pc) = xh_r[q];
                if constexpr (SPLIT) *reinterpret_cast<v4u*>(base + NS * RB + st * RB + 16 * pc) = xl_r[q];
            }
        }
    };
    // the next chunk's operator rows always land in ah_n / al_n and the MFMAs
    // always read ah_r / al_r (fixed arrays keep everything in registers)
    auto load_a_next = [&](int64_t k0) {
#pragma unroll
        for (int sub = 0; sub < NSUB; ++sub)
#pragma unroll
            for (int rt = 0; rt < 2; ++rt) {
                const int64_t row = rowbase + 16 * rt + j;
                if constexpr (PREC == 0) {
                    ah_n[sub][rt] = *reinterpret_cast<const float4*>(Ah + row * G.ld + k0 + 16 * sub + 4 * g);
                } else {
                    const int64_t off = row * G.ld + k0 + 32 * sub + 8 * g;
                    ah_n[sub][rt] = *reinterpret_cast<const AV*>(Ah + off);
                    al_n[sub][rt] = *reinterpret_cast<const AV*>(Al + off);
                }
            }
    };
    auto rotate = [&]() {
#pragma unroll
        for (int sub = 0; sub < NSUB; ++sub)
#pragma unroll
            for (int rt = 0; rt < 2; ++rt) {
                ah_r[sub][rt] = ah_n[sub][rt];
                if constexpr (SPLIT) al_r[sub][rt] = al_n[sub][rt];
            }
    };
    auto compute = [&](int buf) {
        const auto& hi = ah_r;
        const auto& lo = al_r;
        const unsigned char* xs = lds + buf * BUF;
#pragma unroll
        for (int sub = 0; sub < NSUB; ++sub) {
            if constexpr (PREC == 0) {
                float4 b[NST];
#pragma unroll
                for (int st = 0; st < NST; ++st)
                    b[st] = *reinterpret_cast<const float4*>(xs + (16 * st + j) * RB + 4 * (16 * sub + 4 * g));
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int st = 0; st < NST; ++st)
#pragma unroll
                        for (int rt = 0; rt < 2; ++rt) {
                            const float av = q == 0 ? hi[sub][rt].x : q == 1 ? hi[sub][rt].y : q == 2 ? hi[sub][rt].z : hi[sub][rt].w;
                            const float bv = q == 0 ? b[st].x : q == 1 ? b[st].y : q == 2 ? b[st].z : b[st].w;
                            acc[rt][st] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[rt][st], 0, 0, 0);
                        }
            } else {
                const int kk = 32 * sub + 8 * g;
#pragma unroll
                for (int st = 0; st < NST; ++st) {
                    const AV bh = *reinterpret_cast<const AV*>(xs + (16 * st + j) * RB + 2 * kk);
                    const AV bl = *reinterpret_cast<const AV*>(xs + NS * RB + (16 * st + j) * RB + 2 * kk);
                    // three independent products over two accumulators
                    if constexpr (PREC == 1) {
                        acc[0][st] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(hi[sub][0], bh, acc[0][st], 0, 0, 0);
                        acc[1][st] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(hi[sub][1], bh, acc[1][st], 0, 0, 0);
                        acc[0][st] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(hi[sub][0], bl, acc[0][st], 0, 0, 0);
                        acc[1][st] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(hi[sub][1], bl, acc[1][st], 0, 0, 0);
                        acc[0][st] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(lo[sub][0], bh, acc[0][st], 0, 0, 0);
                        acc[1][st] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(lo[sub][1], bh, acc[1][st], 0, 0, 0);
                    } else {
                        acc[0][st] = __builtin_amdgcn_mfma_f32_16x16x32_f16(hi[sub][0], bh, acc[0][st], 0, 0, 0);
                        acc[1][st] = __builtin_amdgcn_mfma_f32_16x16x32_f16(hi[sub][1], bh, acc[1][st], 0, 0, 0);
                        acc[0][st] = __builtin_amdgcn_mfma_f32_16x16x32_f16(hi[sub][0], bl, acc[0][st], 0, 0, 0);
                        acc[1][st] = __builtin_amdgcn_mfma_f32_16x16x32_f16(hi[sub][1], bl, acc[1][st], 0, 0, 0);
                        acc[0][st] = __builtin_amdgcn_mfma_f32_16x16x32_f16(lo[sub][0], bh, acc[0][st], 0, 0, 0);
                        acc[1][st] = __builtin_amdgcn_mfma_f32_16x16x32_f16(lo[sub][1], bh, acc[1][st], 0, 0, 0);
                    }
                }
            }
        }
    };

    if (nch > 0) {
        load_x(kb);
        load_a_next(kb);
        rotate();
        store_x(0);
        __syncthreads();
        for (int c = 0; c < nch; ++c) {
            const bool more = c + 1 < nch;
            const int64_t k1 = kb + static_cast<int64_t>(c + 1) * KC;
            if (more) {
                load_x(k1);
                load_a_next(k1);
            }
            compute(c & 1);
            if (more) {
                store_x((c + 1) & 1);
                rotate();
            }
            __syncthreads();
        }
    }
    // D[4 g + r][j] of tile (rt, st) -> part[split][state 16 st + j][row rowbase + 16 rt + 4 g + r]
    float* out = G.part + static_cast<int64_t>(blockIdx.y) * G.bpad * G.rows;
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
        const int64_t r0 = rowbase + 16 * rt + 4 * g;
        float4 sc = make_float4(1.f, 1.f, 1.f, 1.f);
        if constexpr (PREC == 2) sc = *reinterpret_cast<const float4*>(G.rscale + r0);
#pragma unroll
        for (int st = 0; st < NST; ++st) {
            const v4f v = acc[rt][st];
            *reinterpret_cast<float4*>(out + (16 * st + j) * G.rows + r0) =
                make_float4(v.x * sc.x, v.y * sc.y, v.z * sc.z, v.w * sc.w);
        }
    }
}

// Right operand from the (padded) stage input: (Ms_b / Ms_ref) m, as float32
// or split into hi + lo.
template <int PREC>
__global__ __launch_bounds__(256) void k_prep(int64_t B, int64_t ld, int32_t n, const float* __restrict__ Y,
                                              const float* __restrict__ Ms, float inv_ref,
                                              void* __restrict__ xh, void* __restrict__ xl) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= B * ld) return;
    const int64_t k = i % ld;
    const int64_t b = k / 3;
    const float v = (b < n) ? Y[i] * (Ms[b] * inv_ref) : 0.0f;
    if constexpr (PREC == 0) {
        static_cast<float*>(xh)[i] = v;
    } else if constexpr (PREC == 1) {
        const __bf16 h = static_cast<__bf16>(v);
        static_cast<__bf16*>(xh)[i] = h;
        static_cast<__bf16*>(xl)[i] = static_cast<__bf16>(v - static_cast<float>(h));
    } else {
        const _Float16 h = static_cast<_Float16>(v);
        static_cast<_Float16*>(xh)[i] = h;
        static_cast<_Float16*>(xl)[i] = static_cast<_Float16>(v - static_cast<float>(h));
    }
}

// Sum of the split-K partials in fixed order, then the per-tile finish.
template <Epi MODE>
__global__ __launch_bounds__(256) void k_finish(DevProblem P, const float* __restrict__ part,
                                                int64_t splits, int64_t bpad, int64_t rows,
                                                float scale, const float* __restrict__ X, int64_t sx,
                                                EpiArgs E) {
    const int s = blockIdx.y;
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    double rmax = 0.0, dmax = 0.0;
    if (a < P.n) {
        float h0 = 0.f, h1 = 0.f, h2 = 0.f;
        for (int64_t sp = 0; sp < splits; ++sp) {
            const float* pp = part + (sp * bpad + s) * rows + 3 * static_cast<int64_t>(a);
            h0 += pp[0]; h1 += pp[1]; h2 += pp[2];
        }
        finish_tile<MODE>(P, X, sx, E, s, a, -scale * h0, -scale * h1, -scale * h2, &rmax, &dmax);
    }
    if constexpr (MODE == Epi::DP_LAST) {
        __shared__ double red[2][4];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            rmax = fmax(rmax, __shfl_xor(rmax, off, 64));
            dmax = fmax(dmax, __shfl_xor(dmax, off, 64));
        }
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        if (lane == 0) {
            red[0][wave] = rmax;
            red[1][wave] = dmax;
        }
        __syncthreads();
        if (wave != 0) return;
        rmax = fmax(fmax(red[0][0], red[0][1]), fmax(red[0][2], red[0][3]));
        dmax = fmax(fmax(red[1][0], red[1][1]), fmax(red[1][2], red[1][3]));
        report_partials(E, rmax, dmax, lane);
    }
}

template <int PREC, int NST>
tm_status launch_gemm_t(const GemmArgs& G, int64_t rowblocks, int64_t splits, hipStream_t s) {
    k_gemm<PREC, NST, chunk_for(PREC, NST)>
        <<<dim3(static_cast<unsigned>(rowblocks), static_cast<unsigned>(splits)), 256, 0, s>>>(G);
    TM_TRY_HIP(hipGetLastError());
    return TM_OK;
}

template <int PREC>
tm_status launch_gemm_p(int nst, const GemmArgs& G, int64_t rowblocks, int64_t splits, hipStream_t s) {
    switch (nst) {
        case 1: return launch_gemm_t<PREC, 1>(G, rowblocks, splits, s);
        case 2: return launch_gemm_t<PREC, 2>(G, rowblocks, splits, s);
        case 4: return launch_gemm_t<PREC, 4>(G, rowblocks, splits, s);
        case 8: return launch_gemm_t<PREC, 8>(G, rowblocks, splits, s);
        default: break;
    }
    set_error("batched product: unsupported state-tile count %d", nst);
    return TM_EINVAL;
}

}  // namespace

int gemm_state_tiles(int64_t B) {
    const int64_t t = (B + 15) / 16;
    return t <= 1 ? 1 : t <= 2 ? 2 : t <= 4 ? 4 : 8;
}

int64_t gemm_splits(const Problem* p) {
    const int64_t rowblocks = p->T->rows / kRowsPerBlock;
    const int64_t kchunks = p->T->ld / kKC;
    // about one workgroup per CU (the split-precision kernel holds ~139 KB of LDS)
    int64_t s = (256 + rowblocks - 1) / rowblocks;
    if (s > 1 && rowblocks * s > 256 + rowblocks / 2) s -= 1;
    return std::max<int64_t>(1, std::min<int64_t>(s, std::min<int64_t>(kchunks, 16)));
}

tm_status launch_field_batched(const Problem* p, Epi mode, int64_t B, const float* X,
                               const EpiArgs& e, hipStream_t s) {
    const Tensor* T = p->T;
    Workspace* w = p->ws.get();
    TM_REQUIRE(w && w->part && B <= 128 && w->bpad >= 16 * gemm_state_tiles(B), TM_EINVAL,
               "batched product: workspace not prepared for %lld states", static_cast<long long>(B));
    TM_REQUIRE(T->ld % kKC == 0 && T->rows % kRowsPerBlock == 0 && T->rows >= T->ld, TM_EINVAL,
               "batched product: operator extent %lld x %lld is not a whole number of tiles",
               static_cast<long long>(T->rows), static_cast<long long>(T->ld));
    const int prec = T->prec == TM_PREC_FP32 ? 0 : T->prec == TM_PREC_BF16X3 ? 1 : 2;
    const int64_t ld = T->ld;
    // right operand
    const void* xh = X;
    const void* xl = nullptr;
    if (prec != 0 || !p->uniform_ms) {
        const int64_t cnt = B * ld;
        const unsigned grid = static_cast<unsigned>((cnt + 255) / 256);
        const float inv = static_cast<float>(1.0 / p->ms_ref);
        if (prec == 0)
            k_prep<0><<<grid, 256, 0, s>>>(B, ld, static_cast<int32_t>(p->n), X, p->Ms, inv, w->xh, nullptr);
        else if (prec == 1)
            k_prep<1><<<grid, 256, 0, s>>>(B, ld, static_cast<int32_t>(p->n), X, p->Ms, inv, w->xh, w->xl);
        else
            k_prep<2><<<grid, 256, 0, s>>>(B, ld, static_cast<int32_t>(p->n), X, p->Ms, inv, w->xh, w->xl);
        TM_TRY_HIP(hipGetLastError());
        xh = w->xh;
        xl = w->xl;
    }
    GemmArgs G;
    G.ld = ld;
    G.bpad = w->bpad;
    G.Ahi = T->data;
    G.Alo = T->lo;
    G.rscale = T->rscale;
    G.Xhi = xh;
    G.Xlo = xl;
    G.part = w->part;
    G.rows = T->rows;
    const int64_t splits = w->part_splits;
    const int nst = gemm_state_tiles(B);
    G.kper = round_up((ld + splits - 1) / splits, chunk_for(prec, nst));
    const int64_t used_splits = (ld + G.kper - 1) / G.kper;
    const int64_t rowblocks = T->rows / kRowsPerBlock;
    tm_status st = prec == 0   ? launch_gemm_p<0>(nst, G, rowblocks, used_splits, s)
                   : prec == 1 ? launch_gemm_p<1>(nst, G, rowblocks, used_splits, s)
                               : launch_gemm_p<2>(nst, G, rowblocks, used_splits, s);
    if (st != TM_OK) return st;
    // X holds (Ms_b / Ms_ref) m (or m itself when Ms is uniform): H_d = -Ms_ref C
    const float scale = static_cast<float>(p->ms_ref);
    const DevProblem P = p->dev();
    const dim3 grid(static_cast<unsigned>((p->n + 255) / 256), static_cast<unsigned>(B));
    const int64_t sx = 3 * p->np;
    switch (mode) {
        case Epi::HD: k_finish<Epi::HD><<<grid, 256, 0, s>>>(P, w->part, used_splits, w->bpad, T->rows, scale, X, sx, e); break;
        case Epi::HEFF: k_finish<Epi::HEFF><<<grid, 256, 0, s>>>(P, w->part, used_splits, w->bpad, T->rows, scale, X, sx, e); break;
        case Epi::DMDT: k_finish<Epi::DMDT><<<grid, 256, 0, s>>>(P, w->part, used_splits, w->bpad, T->rows, scale, X, sx, e); break;
        case Epi::STAGE: k_finish<Epi::STAGE><<<grid, 256, 0, s>>>(P, w->part, used_splits, w->bpad, T->rows, scale, X, sx, e); break;
        case Epi::RK4_FINAL: k_finish<Epi::RK4_FINAL><<<grid, 256, 0, s>>>(P, w->part, used_splits, w->bpad, T->rows, scale, X, sx, e); break;
        case Epi::DP_LAST: k_finish<Epi::DP_LAST><<<grid, 256, 0, s>>>(P, w->part, used_splits, w->bpad, T->rows, scale, X, sx, e); break;
    }
    TM_TRY_HIP(hipGetLastError());
    return TM_OK;
}

}  // namespace tmag
