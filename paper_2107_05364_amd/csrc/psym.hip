// Pair-symmetric demag operator (PSYM6 / PSYM4) for meshes of identical tiles.
//
// When every tile has the same edges the tensor of tile b at the centre of
// tile a depends only on the centre offset and is even in it, so
// N^{ab} = N^{ba}; with the symmetry of each 3x3 block this is the symmetry
// the paper invokes to store roughly half of the operator (Sec. 3.2).  The
// operator is cut into TS x TS-block tiles (TS = kPsTile) and only the tile
// pairs I <= J are stored ([pairs][6][TS][TS] float32, a diagonal tile in
// full).  PSYM4, for a single layer of tiles (one z for every centre), keeps
// four planes: the xz and yz components are odd in the z offset and vanish.
//
// Product, two launches per field evaluation:
//  * k_psym_tiles: one workgroup per tile pair (and group of states) reads its
//    tile once and forms both uses of it for each state: the row sums  sum_b N^{ab} (Ms m)_b  for the
//    targets a of tile I, and for I < J the column sums
//    sum_a N^{ab} (Ms m)_a = sum_a N^{ba} (Ms m)_a  for the targets b of
//    tile J.  Each lands in its own slot part[s][K][j][TS][3] (K = the target
//    tile, j = the other tile), so every slot has exactly one writer.
//  * k_psym_finish: one workgroup per (target tile K, state) adds the nt
//    slots of K (a fixed order: results do not depend on scheduling or on
//    the batch) and completes the right-hand side and the stage for its TS
//    tiles; the local field terms were folded into the diagonal slot by the
//    tile pass.
// Streamed bytes: 24 B x TS^2 per stored tile pair, i.e. about 12 N^2 + 12 N TS
// against 24 N^2 for SYM6 (PSYM4: 16 B x TS^2, about 8 N^2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "common.h"
#include "epilogue.h"

namespace tmag {
namespace {

constexpr int TS = kPsTile;
constexpr int TB = kPsTile * kPsTile;
constexpr int kTileThreads = 256;  // tile pass workgroup
constexpr int RG = kTileThreads / TS;  // row groups of a workgroup (one column per lane)
constexpr int RPT = TS / RG;       // rows per thread
static_assert(TS * RG == kTileThreads && RPT * RG == TS, "tile size must divide the workgroup");
// reduction + epilogue workgroup: kFinishGroups groups of kFinishPos threads,
// each thread adding kFinishLoads float4 of its group's slots per round
constexpr int kFinishThreads = 256;
constexpr int kFinishPos = 3 * TS / 4;   // float4 per slot
constexpr int kFinishGroups = 10;
constexpr int kFinishLoads = 8;
static_assert(kFinishGroups * kFinishPos <= kFinishThreads && kFinishThreads >= 64 && 3 * TS % 4 == 0,
              "finish workgroup shape");
typedef float f4 __attribute__((ext_vector_type(4)));

template <bool NTL>
__device__ inline float ldt(const float* p) {
    if constexpr (NTL) return __builtin_nontemporal_load(p);
    else return *p;
}

// Index of tile pair (I, J), I <= J, in the pair table: the nt diagonal
// pairs first, then the pairs I < J in row-major order.
inline int64_t pair_index(int64_t I, int64_t J, int64_t nt) {
    return I == J ? I : nt + I * (nt - 1) - I * (I - 1) / 2 + (J - I - 1);
}

// One workgroup per tile pair and state (MULTI = false: the grid has B rows)
// or per tile pair and group of states (MULTI = true: states s = blockIdx.y,
// blockIdx.y + gridDim.y, ..., so that a batch streams each tile once per
// group).  The workgroup reads its tile once and applies it to its states.
// Thread t takes column b = t % TS of the tile and rows rg RPT .. rg RPT +
// RPT - 1 (rg = t / TS): each row's components are coalesced loads.  Per
// state the Ms-scaled inputs of the two tiles are staged in LDS (one
// coalesced load per component), the row sums go through LDS to a sum over
// the TS columns (four interleaved partial sums), the column sums through LDS
// to a sum over the RG groups (both in a fixed order, the same for either
// grid: results do not depend on the batch).
//
// LOCALF: the workgroups of diagonal pairs (I == J) also evaluate the local
// field terms (exchange, anisotropy, applied field) of their TS tiles --
// issued before the tile's products, so that the dependent neighbour loads
// overlap the tile loads, and dispatched first (diagonal pairs lead the pair
// table) -- and subtract them from their own slot, so that minus the slot sum
// is the whole effective field and the finish kernel has no dependent loads
// left.
// NP = 6: planes (xx, xy, xz, yy, yz, zz); NP = 4 (a single layer): (xx, xy,
// yy, zz), with xz = yz = 0.
template <bool STEPPING, bool LOCALF, bool NTL, int NP, bool MULTI>
__global__ __launch_bounds__(kTileThreads) void k_psym_tiles(DevProblem P, const float* __restrict__ tiles,
                                                    const int32_t* __restrict__ pairs, int64_t nt,
                                                    const float* __restrict__ Ms, const float* __restrict__ X,
                                                    int64_t sx, const double* __restrict__ h,
                                                    const float* __restrict__ Ha, float* __restrict__ part,
                                                    int64_t B) {
    const int64_t p = blockIdx.x;
    const int t = threadIdx.x;
    const int b = t % TS, rg = t / TS;
    // frozen states read no operator (a batch may hold many of them): a
    // workgroup whose states are all frozen stops before loading its tile
    if (STEPPING) {
        bool live = false;
        if constexpr (MULTI) {
            for (int64_t s = blockIdx.y; s < B && !live; s += gridDim.y) live = h[s] != 0.0;
        } else {
            live = h[blockIdx.y] != 0.0;
        }
        if (!live) return;
    }
    const float* tile = tiles + p * NP * TB;
    float v[RPT][NP];
#pragma unroll
    for (int i = 0; i < RPT; ++i)
#pragma unroll
        for (int c = 0; c < NP; ++c) v[i][c] = ldt<NTL>(tile + c * TB + (RPT * rg + i) * TS + b);
    const int64_t I = pairs[2 * p], J = pairs[2 * p + 1];
    __shared__ float rred[TS][3][TS + 1];  // row sums before the column reduction
    __shared__ float cred[RG][TS][3];      // column sums per row group
    __shared__ float hl[TS][3];            // local field terms (diagonal pairs)
    __shared__ float xs[2][TS][3];         // Ms-scaled stage input of tile I (rows) and tile J (columns)
    // the products of state s with the tile in registers (slots of s written)
    auto one_state = [&](int64_t s) {
        const float* x = X + s * sx;
        // the Ms-scaled inputs of the pair's 2 x TS tiles, staged once: one
        // coalesced load per component instead of a load per thread and use
        if (t < 6 * TS) {
            const int half = t / (3 * TS), r = t % (3 * TS);
            const int64_t q0 = TS * (half ? J : I);
            xs[half][r / 3][r % 3] = x[3 * q0 + r] * Ms[q0 + r / 3];
        }
        if (LOCALF && I == J && t < TS) {
            const int64_t a = TS * I + t;
            float H0 = 0.0f, H1 = 0.0f, H2 = 0.0f;
            if (a < P.n)
                add_local_field(P, x, Ha, static_cast<int>(s), static_cast<int>(a), x[3 * a], x[3 * a + 1],
                                x[3 * a + 2], H0, H1, H2);
            hl[t][0] = H0;
            hl[t][1] = H1;
            hl[t][2] = H2;
        }
        __syncthreads();
        const float xb0 = xs[1][b][0], xb1 = xs[1][b][1], xb2 = xs[1][b][2];
        float c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            const int al = RPT * rg + i;
            const float xa0 = xs[0][al][0], xa1 = xs[0][al][1], xa2 = xs[0][al][2];
            const float v0 = v[i][0], v1 = v[i][1];
            const float v2 = NP == 6 ? v[i][2] : 0.0f, v3 = v[i][NP == 6 ? 3 : 2];
            const float v4 = NP == 6 ? v[i][4] : 0.0f, v5 = v[i][NP - 1];
            rred[al][0][b] = v0 * xb0 + v1 * xb1 + v2 * xb2;
            rred[al][1][b] = v1 * xb0 + v3 * xb1 + v4 * xb2;
            rred[al][2][b] = v2 * xb0 + v4 * xb1 + v5 * xb2;
            c0 += v0 * xa0 + v1 * xa1 + v2 * xa2;
            c1 += v1 * xa0 + v3 * xa1 + v4 * xa2;
            c2 += v2 * xa0 + v4 * xa1 + v5 * xa2;
        }
        cred[rg][b][0] = c0;
        cred[rg][b][1] = c1;
        cred[rg][b][2] = c2;
        __syncthreads();
        if (t < 3 * TS) {
            const int r = t / 3, c = t % 3;
            // four interleaved partial sums (columns l mod 4), then a fixed
            // pairwise order: a quarter of the dependent adds
            float a4[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int l = 0; l < TS; ++l) a4[l % 4] += rred[r][c][l];
            float acc = (a4[0] + a4[1]) + (a4[2] + a4[3]);
            if (LOCALF && I == J) acc -= hl[r][c];
            // the slots are read once, by the finish (on another XCD): streaming stores
            __builtin_nontemporal_store(acc, part + ((s * nt + I) * nt + J) * (3 * TS) + t);
            if (I != J) {
                float cs = 0.0f;
#pragma unroll
                for (int q = 0; q < RG; ++q) cs += cred[q][r][c];
                __builtin_nontemporal_store(cs, part + ((s * nt + J) * nt + I) * (3 * TS) + t);
            }
        }
    };
    if constexpr (MULTI) {
        bool first = true;
        for (int64_t s = blockIdx.y; s < B; s += gridDim.y) {
            if (STEPPING && h[s] == 0.0) continue;
            if (!first) __syncthreads();  // the previous state's sums have been read
            first = false;
            one_state(s);
        }
    } else {
        one_state(blockIdx.y);
    }
}

// By default operators larger than the Infinity Cache are streamed with
// nontemporal loads (each tile is read once per evaluation and cannot stay
// cached anyway).  Which loads are faster below that size varies (the film
// at N = 2500 streams faster with nontemporal loads, at N = 4900 in four
// planes slower), so tm_problem_tune times both on the caller's problem.
constexpr int64_t kPsymStreamBytes = 192ll << 20;

template <bool STEPPING, bool LOCALF, int NP>
inline void launch_tiles_np(dim3 grid, hipStream_t st, bool nt_loads, const DevProblem& P, const float* tiles,
                            const int32_t* pairs, int64_t nt, const float* Ms, const float* X, int64_t sx,
                            const double* h, const float* Ha, float* part, int64_t B) {
    // one state per workgroup when the grid has a row per state
    const bool multi = grid.y < B;
    if (nt_loads) {
        if (multi)
            launch_op(k_psym_tiles<STEPPING, LOCALF, true, NP, true>, grid, dim3(kTileThreads), st, P, tiles, pairs,
                      nt, Ms, X, sx, h, Ha, part, B);
        else
            launch_op(k_psym_tiles<STEPPING, LOCALF, true, NP, false>, grid, dim3(kTileThreads), st, P, tiles, pairs,
                      nt, Ms, X, sx, h, Ha, part, B);
    } else {
        if (multi)
            launch_op(k_psym_tiles<STEPPING, LOCALF, false, NP, true>, grid, dim3(kTileThreads), st, P, tiles,
                      pairs, nt, Ms, X, sx, h, Ha, part, B);
        else
            launch_op(k_psym_tiles<STEPPING, LOCALF, false, NP, false>, grid, dim3(kTileThreads), st, P, tiles,
                      pairs, nt, Ms, X, sx, h, Ha, part, B);
    }
}

// Grid of the tile pass for B states: one workgroup per tile pair and group
// of states.  A pair's tile is read once per group, so the fewer groups the
// fewer operator bytes; the states are split over several groups only while
// the pairs alone leave the 256 CUs short of work (kTileWorkgroups).
constexpr int64_t kTileWorkgroups = 1024;
dim3 tile_grid(const Tensor* T, int64_t B) {
    const int64_t groups = std::min<int64_t>(B, std::max<int64_t>(1, (kTileWorkgroups + T->npairs - 1) / T->npairs));
    return dim3(static_cast<unsigned>(T->npairs), static_cast<unsigned>(groups));
}

template <bool STEPPING, bool LOCALF>
inline void launch_tiles(const Tensor* T, bool nt_loads, int64_t B, hipStream_t st, const DevProblem& P,
                         const float* Ms, const float* X, int64_t sx, const double* h, const float* Ha,
                         float* part) {
    const float* tiles = static_cast<const float*>(T->data);
    const dim3 grid = tile_grid(T, B);
    if (T->layout == TM_LAYOUT_PSYM4)
        launch_tiles_np<STEPPING, LOCALF, 4>(grid, st, nt_loads, P, tiles, T->pairs, T->nt, Ms, X, sx, h, Ha, part, B);
    else
        launch_tiles_np<STEPPING, LOCALF, 6>(grid, st, nt_loads, P, tiles, T->pairs, T->nt, Ms, X, sx, h, Ha, part, B);
}

// One workgroup per (target tile K, state): the nt slots of K are contiguous
// ([nt][TS][3] floats, kFinishPos float4 each).  Thread (g, pos) = (t /
// kFinishPos, t % kFinishPos), g < kFinishGroups, adds float4 number pos of
// the slots j = g, g + kFinishGroups, ... in ascending j, kFinishLoads
// independent 16-byte loads per round (one round for nt <= 80; past the last
// slot the load repeats it and the value is not added: no branches between
// the loads); the group sums go through LDS and the first TS lanes of wave 0
// add them in order g = 0 .. kFinishGroups - 1 per tile and run the epilogue.
// The slots are requested before anything else (they depend only on K and
// s), the epilogue's own inputs next; a frozen state then stops or skips.
template <Epi MODE>
__global__ __launch_bounds__(kFinishThreads) void k_psym_finish(DevProblem P, const float* __restrict__ part,
                                                                int64_t nt, const float* X, int64_t sx, EpiArgs E) {
    constexpr bool STEPPING = MODE == Epi::STAGE || MODE == Epi::RK4_FINAL || MODE == Epi::DP_LAST;
    constexpr int U = kFinishLoads, G = kFinishGroups;
    const int64_t K = blockIdx.x;
    const int s = blockIdx.y;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int pos = t % kFinishPos, g = t / kFinishPos;
    const bool adds = g < G;
    rk4_last_stage_control<MODE>(E);
    __shared__ f4 gs[G][kFinishPos];
    const f4* src = reinterpret_cast<const f4*>(part + (static_cast<int64_t>(s) * nt + K) * nt * (3 * TS)) + pos;
    f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    int64_t j = g;
    f4 v[U];
    if (adds) {
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = src[min(j + u * G, nt - 1) * kFinishPos];
    }
    const int64_t a = TS * K + lane;
    const bool mine0 = wave == 0 && lane < TS && a < P.n;
    EpiIn in;
    if (mine0) epi_load<MODE>(X, sx, E, s, static_cast<int>(a), in);
    bool frozen = false;
    if constexpr (STEPPING) frozen = E.h[s] == 0.0;
    if constexpr (MODE == Epi::STAGE || MODE == Epi::RK4_FINAL) {
        if (frozen) return;
    }
    if (adds) {
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (j + u * G < nt) acc += v[u];
        j += U * G;
        if (!frozen) {
            for (; j < nt; j += U * G) {
#pragma unroll
                for (int u = 0; u < U; ++u) v[u] = src[min(j + u * G, nt - 1) * kFinishPos];
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (j + u * G < nt) acc += v[u];
            }
        }
        gs[g][pos] = acc;
    }
    __syncthreads();
    if (wave != 0) return;
    double rmax = 0.0, dmax = 0.0;
    if (mine0 && !frozen) {
        const float* gf = reinterpret_cast<const float*>(&gs[0][0]);
        float hx = 0.0f, hy = 0.0f, hz = 0.0f;
#pragma unroll
        for (int g2 = 0; g2 < G; ++g2) {
            hx += gf[g2 * 3 * TS + 3 * lane];
            hy += gf[g2 * 3 * TS + 3 * lane + 1];
            hz += gf[g2 * 3 * TS + 3 * lane + 2];
        }
        epi_compute<MODE>(P, sx, E, s, static_cast<int>(a), in, -hx, -hy, -hz, &rmax, &dmax);
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

template <Epi MODE>
void launch_psym_t(const DevProblem& P, const Tensor* T, bool nt_loads, const float* Ms, float* part, int64_t B,
                   const float* X, int64_t sx, const EpiArgs& e, hipStream_t s) {
    constexpr bool STEPPING = MODE == Epi::STAGE || MODE == Epi::RK4_FINAL || MODE == Epi::DP_LAST;
    constexpr bool LOCALF = MODE != Epi::HD;
    launch_tiles<STEPPING, LOCALF>(T, nt_loads, B, s, P, Ms, X, sx, e.h, e.Ha, part);
    const dim3 g2(static_cast<unsigned>(T->nt), static_cast<unsigned>(B));
    k_psym_finish<MODE><<<g2, kFinishThreads, 0, s>>>(P, part, T->nt, X, sx, e);
}

// Operator loads of the tile pass: the problem's choice (tm_problem_tune),
// else nontemporal beyond the Infinity Cache.
bool psym_nt_loads(const Problem* p) {
    return p->psym_nt >= 0 ? p->psym_nt == 1 : p->T->bytes > kPsymStreamBytes;
}

}  // namespace

int64_t psym_partial_floats(const Tensor* T, int64_t B) { return B * T->nt * T->nt * 3 * TS; }

tm_status launch_psym_tiles(const Problem* p, int64_t B, const float* X, const double* h, const float* Ha,
                            hipStream_t s) {
    const Tensor* T = p->T;
    Workspace* w = p->ws.get();
    TM_REQUIRE(is_psym(T->layout) && w && w->part && w->B >= B, TM_EINVAL,
               "pair-symmetric tile pass: not prepared");
    launch_tiles<true, true>(T, psym_nt_loads(p), B, s, p->dev(), p->Ms, X, 3 * p->np, h, Ha, w->part);
    TM_TRY_HIP(hipGetLastError());
    return TM_OK;
}

tm_status launch_field_psym(const Problem* p, Epi mode, int64_t B, const float* X, const EpiArgs& e,
                            hipStream_t s) {
    Workspace* w = p->ws.get();
    TM_REQUIRE(w && w->part && w->B >= B, TM_EINVAL,
               "pair-symmetric field evaluation: workspace not prepared for %lld states",
               static_cast<long long>(B));
    return launch_field_psym_slots(p, mode, B, X, e, w->part, s);
}

tm_status launch_field_psym_slots(const Problem* p, Epi mode, int64_t B, const float* X, const EpiArgs& e,
                                  float* part, hipStream_t s) {
    const Tensor* T = p->T;
    TM_REQUIRE(is_psym(T->layout) && T->pairs && T->data, TM_EINVAL,
               "pair-symmetric field evaluation needs a PSYM6 or PSYM4 operator");
    TM_REQUIRE(part && B >= 1 && B <= 65535, TM_EINVAL,
               "pair-symmetric field evaluation: no slot buffer or bad batch %lld", static_cast<long long>(B));
    TM_REQUIRE(p->np >= TS * T->nt, TM_EINVAL, "pair-symmetric field evaluation: state padding too small");
    const DevProblem P = p->dev();
    const int64_t sx = 3 * p->np;
    const bool nt = psym_nt_loads(p);
    switch (mode) {
        case Epi::HD: launch_psym_t<Epi::HD>(P, T, nt, p->Ms, part, B, X, sx, e, s); break;
        case Epi::HEFF: launch_psym_t<Epi::HEFF>(P, T, nt, p->Ms, part, B, X, sx, e, s); break;
        case Epi::DMDT: launch_psym_t<Epi::DMDT>(P, T, nt, p->Ms, part, B, X, sx, e, s); break;
        case Epi::STAGE: launch_psym_t<Epi::STAGE>(P, T, nt, p->Ms, part, B, X, sx, e, s); break;
        case Epi::RK4_FINAL: launch_psym_t<Epi::RK4_FINAL>(P, T, nt, p->Ms, part, B, X, sx, e, s); break;
        case Epi::DP_LAST: launch_psym_t<Epi::DP_LAST>(P, T, nt, p->Ms, part, B, X, sx, e, s); break;
    }
    TM_TRY_HIP(hipGetLastError());
    return TM_OK;
}

tm_status psym_rows(const Tensor* T, int64_t a0, int64_t count, double* out) {
    const int64_t n = T->n, nt = T->nt;
    const int NP = psym_planes(T->layout);
    std::vector<float> tile(NP * TB);
    // plane of each of the 9 components (-1: zero, not stored)
    static const int comp6[9] = {0, 1, 2, 1, 3, 4, 2, 4, 5};
    static const int comp4[9] = {0, 1, -1, 1, 2, -1, -1, -1, 3};
    const int* comp = NP == 4 ? comp4 : comp6;
    for (int64_t ta = a0 / TS; ta <= (a0 + count - 1) / TS; ++ta) {
        for (int64_t tb = 0; tb < nt; ++tb) {
            const bool upper = ta <= tb;
            const int64_t pidx = upper ? pair_index(ta, tb, nt) : pair_index(tb, ta, nt);
            TM_TRY_HIP(hipMemcpy(tile.data(), static_cast<const float*>(T->data) + pidx * NP * TB,
                                 NP * TB * sizeof(float), hipMemcpyDeviceToHost));
            for (int64_t al = 0; al < TS; ++al) {
                const int64_t a = TS * ta + al;
                if (a < a0 || a >= a0 + count) continue;
                for (int64_t bl = 0; bl < TS; ++bl) {
                    const int64_t b = TS * tb + bl;
                    if (b >= n) break;
                    // N^{ab} from tile (ta, tb) at (al, bl), or N^{ba} = N^{ab} from (tb, ta) at (bl, al)
                    const int64_t e = upper ? al * TS + bl : bl * TS + al;
                    for (int k = 0; k < 9; ++k)
                        out[((a - a0) * n + b) * 9 + k] = comp[k] < 0 ? 0.0 : tile[comp[k] * TB + e];
                }
            }
        }
    }
    return TM_OK;
}

}  // namespace tmag
