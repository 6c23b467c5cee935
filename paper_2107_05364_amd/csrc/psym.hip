// Pair-symmetric demag operator (PSYM6) for meshes of identical tiles.
//
// When every tile has the same edges the tensor of tile b at the centre of
// tile a depends only on the centre offset and is even in it, so
// N^{ab} = N^{ba}; with the symmetry of each 3x3 block this is the symmetry
// the paper invokes to store roughly half of the operator (Sec. 3.2).  The
// operator is cut into 64 x 64-block tiles and only the tile pairs I <= J are
// stored ([pairs][6][64][64] float32, a diagonal tile in full).
//
// Product, two launches per field evaluation:
//  * k_psym_tiles: one workgroup per (tile pair, state) reads its tile once
//    and forms both uses of it: the row sums  sum_b N^{ab} (Ms m)_b  for the
//    targets a of tile I, and for I < J the column sums
//    sum_a N^{ab} (Ms m)_a = sum_a N^{ba} (Ms m)_a  for the targets b of
//    tile J.  Each lands in its own slot part[s][K][j][64][3] (K = the target
//    tile, j = the other tile), so every slot has exactly one writer.
//  * k_psym_finish: one workgroup per (target tile K, state) adds the nt
//    slots of K in ascending j (a fixed order: results do not depend on
//    scheduling or on the batch) and runs the fused epilogue for its 64
//    tiles.
// Streamed bytes: 24 B x 4096 per stored tile pair, i.e. about 12 N^2 + 12 N x 64
// against 24 N^2 for SYM6.
#include <hip/hip_runtime.h>

#include <vector>

#include "common.h"
#include "epilogue.h"

namespace tmag {
namespace {

constexpr int TS = kPsTile;
constexpr int TB = kPsTile * kPsTile;
constexpr int kRowsPerWave = TS / 4;

// Index of tile pair (I, J), I <= J, in row-major upper-triangle order.
inline int64_t pair_index(int64_t I, int64_t J, int64_t nt) { return I * nt - I * (I - 1) / 2 + (J - I); }

template <bool STEPPING>
__global__ __launch_bounds__(256) void k_psym_tiles(const float* __restrict__ tiles,
                                                    const int32_t* __restrict__ pairs, int64_t nt,
                                                    const float* __restrict__ Ms, const float* __restrict__ X,
                                                    int64_t sx, const double* __restrict__ h,
                                                    float* __restrict__ part) {
    const int64_t p = blockIdx.x;
    const int64_t s = blockIdx.y;
    if (STEPPING && h[s] == 0.0) return;  // frozen state: its slots are not read
    const int64_t I = pairs[2 * p], J = pairs[2 * p + 1];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __shared__ float rred[TS][3][TS + 1];  // row sums before the lane reduction
    __shared__ float cred[4][TS][3];       // column sums per wave
    const float* x = X + s * sx;
    const int64_t bg = TS * J + lane;
    const float msb = Ms[bg];
    const float xb0 = x[3 * bg] * msb, xb1 = x[3 * bg + 1] * msb, xb2 = x[3 * bg + 2] * msb;
    const float* tile = tiles + p * 6 * TB;
    float c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
#pragma unroll 4
    for (int i = 0; i < kRowsPerWave; ++i) {
        const int al = kRowsPerWave * w + i;
        const int64_t ag = TS * I + al;
        const float msa = Ms[ag];
        const float xa0 = x[3 * ag] * msa, xa1 = x[3 * ag + 1] * msa, xa2 = x[3 * ag + 2] * msa;
        const int off = al * TS + lane;
        const float v0 = tile[off], v1 = tile[TB + off], v2 = tile[2 * TB + off];
        const float v3 = tile[3 * TB + off], v4 = tile[4 * TB + off], v5 = tile[5 * TB + off];
        rred[al][0][lane] = v0 * xb0 + v1 * xb1 + v2 * xb2;
        rred[al][1][lane] = v1 * xb0 + v3 * xb1 + v4 * xb2;
        rred[al][2][lane] = v2 * xb0 + v4 * xb1 + v5 * xb2;
        c0 += v0 * xa0 + v1 * xa1 + v2 * xa2;
        c1 += v1 * xa0 + v3 * xa1 + v4 * xa2;
        c2 += v2 * xa0 + v4 * xa1 + v5 * xa2;
    }
    cred[w][lane][0] = c0;
    cred[w][lane][1] = c1;
    cred[w][lane][2] = c2;
    __syncthreads();
    const int t = threadIdx.x;
    if (t < 3 * TS) {
        const int r = t / 3, c = t % 3;
        float acc = 0.0f;
#pragma unroll 8
        for (int l = 0; l < TS; ++l) acc += rred[r][c][l];
        part[((s * nt + I) * nt + J) * (3 * TS) + t] = acc;
        if (I != J) {
            const float cs = ((cred[0][r][c] + cred[1][r][c]) + cred[2][r][c]) + cred[3][r][c];
            part[((s * nt + J) * nt + I) * (3 * TS) + t] = cs;
        }
    }
}

template <Epi MODE>
__global__ __launch_bounds__(256) void k_psym_finish(DevProblem P, const float* __restrict__ part, int64_t nt,
                                                     const float* X, int64_t sx, EpiArgs E) {
    constexpr bool STEPPING = MODE == Epi::STAGE || MODE == Epi::RK4_FINAL || MODE == Epi::DP_LAST;
    const int64_t K = blockIdx.x;
    const int s = blockIdx.y;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    bool frozen = false;
    if constexpr (STEPPING) frozen = E.h[s] == 0.0;
    if constexpr (MODE == Epi::STAGE || MODE == Epi::RK4_FINAL) {
        if (frozen) return;
    }
    __shared__ float hb[3 * TS];
    const int t = threadIdx.x;
    if (!frozen && t < 3 * TS) {
        const float* src = part + (static_cast<int64_t>(s) * nt + K) * nt * (3 * TS) + t;
        float acc = 0.0f;
        for (int64_t j = 0; j < nt; ++j) acc += src[j * (3 * TS)];
        hb[t] = -acc;
    }
    __syncthreads();
    if (wave != 0) return;
    double rmax = 0.0, dmax = 0.0;
    const int64_t a = TS * K + lane;
    if (!frozen && a < P.n)
        finish_tile<MODE>(P, X, sx, E, s, a, hb[3 * lane], hb[3 * lane + 1], hb[3 * lane + 2], &rmax, &dmax);
    if constexpr (MODE == Epi::DP_LAST) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            rmax = fmax(rmax, __shfl_xor(rmax, off, 64));
            dmax = fmax(dmax, __shfl_xor(dmax, off, 64));
        }
        report_partials(E, rmax, dmax, lane);
    }
}

template <Epi MODE>
void launch_psym_t(const DevProblem& P, const Tensor* T, const float* Ms, float* part, int64_t B,
                   const float* X, int64_t sx, const EpiArgs& e, hipStream_t s) {
    constexpr bool STEPPING = MODE == Epi::STAGE || MODE == Epi::RK4_FINAL || MODE == Epi::DP_LAST;
    const dim3 g1(static_cast<unsigned>(T->npairs), static_cast<unsigned>(B));
    k_psym_tiles<STEPPING><<<g1, 256, 0, s>>>(static_cast<const float*>(T->data), T->pairs, T->nt, Ms, X, sx,
                                              e.h, part);
    const dim3 g2(static_cast<unsigned>(T->nt), static_cast<unsigned>(B));
    k_psym_finish<MODE><<<g2, 256, 0, s>>>(P, part, T->nt, X, sx, e);
}

}  // namespace

int64_t psym_partial_floats(const Tensor* T, int64_t B) { return B * T->nt * T->nt * 3 * TS; }

tm_status launch_psym_tiles(const Problem* p, int64_t B, const float* X, const double* h, hipStream_t s) {
    const Tensor* T = p->T;
    Workspace* w = p->ws.get();
    TM_REQUIRE(T->layout == TM_LAYOUT_PSYM6 && w && w->part && w->B >= B, TM_EINVAL,
               "pair-symmetric tile pass: not prepared");
    const dim3 g1(static_cast<unsigned>(T->npairs), static_cast<unsigned>(B));
    k_psym_tiles<true><<<g1, 256, 0, s>>>(static_cast<const float*>(T->data), T->pairs, T->nt, p->Ms, X,
                                          3 * p->np, h, w->part);
    TM_TRY_HIP(hipGetLastError());
    return TM_OK;
}

tm_status launch_field_psym(const Problem* p, Epi mode, int64_t B, const float* X, const EpiArgs& e,
                            hipStream_t s) {
    const Tensor* T = p->T;
    Workspace* w = p->ws.get();
    TM_REQUIRE(T->layout == TM_LAYOUT_PSYM6 && T->pairs && T->data, TM_EINVAL,
               "pair-symmetric field evaluation needs a PSYM6 operator");
    TM_REQUIRE(w && w->part && w->B >= B && B >= 1 && B <= 65535, TM_EINVAL,
               "pair-symmetric field evaluation: workspace not prepared for %lld states",
               static_cast<long long>(B));
    TM_REQUIRE(p->np >= TS * T->nt, TM_EINVAL, "pair-symmetric field evaluation: state padding too small");
    const DevProblem P = p->dev();
    const int64_t sx = 3 * p->np;
    switch (mode) {
        case Epi::HD: launch_psym_t<Epi::HD>(P, T, p->Ms, w->part, B, X, sx, e, s); break;
        case Epi::HEFF: launch_psym_t<Epi::HEFF>(P, T, p->Ms, w->part, B, X, sx, e, s); break;
        case Epi::DMDT: launch_psym_t<Epi::DMDT>(P, T, p->Ms, w->part, B, X, sx, e, s); break;
        case Epi::STAGE: launch_psym_t<Epi::STAGE>(P, T, p->Ms, w->part, B, X, sx, e, s); break;
        case Epi::RK4_FINAL: launch_psym_t<Epi::RK4_FINAL>(P, T, p->Ms, w->part, B, X, sx, e, s); break;
        case Epi::DP_LAST: launch_psym_t<Epi::DP_LAST>(P, T, p->Ms, w->part, B, X, sx, e, s); break;
    }
    TM_TRY_HIP(hipGetLastError());
    return TM_OK;
}

tm_status psym_rows(const Tensor* T, int64_t a0, int64_t count, double* out) {
    const int64_t n = T->n, nt = T->nt;
    std::vector<float> tile(6 * TB);
    static const int comp[9] = {0, 1, 2, 1, 3, 4, 2, 4, 5};
    for (int64_t ta = a0 / TS; ta <= (a0 + count - 1) / TS; ++ta) {
        for (int64_t tb = 0; tb < nt; ++tb) {
            const bool upper = ta <= tb;
            const int64_t pidx = upper ? pair_index(ta, tb, nt) : pair_index(tb, ta, nt);
            TM_TRY_HIP(hipMemcpy(tile.data(), static_cast<const float*>(T->data) + pidx * 6 * TB,
                                 6 * TB * sizeof(float), hipMemcpyDeviceToHost));
            for (int64_t al = 0; al < TS; ++al) {
                const int64_t a = TS * ta + al;
                if (a < a0 || a >= a0 + count) continue;
                for (int64_t bl = 0; bl < TS; ++bl) {
                    const int64_t b = TS * tb + bl;
                    if (b >= n) break;
                    // N^{ab} from tile (ta, tb) at (al, bl), or N^{ba} = N^{ab} from (tb, ta) at (bl, al)
                    const int64_t e = upper ? al * TS + bl : bl * TS + al;
                    for (int k = 0; k < 9; ++k) out[((a - a0) * n + b) * 9 + k] = tile[comp[k] * TB + e];
                }
            }
        }
    }
    return TM_OK;
}

}  // namespace tmag
