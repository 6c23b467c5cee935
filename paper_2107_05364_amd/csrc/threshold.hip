// Thresholded demag operator (paper Sec. 4.3.1): the smallest fraction of
// the nonzero tensor entries is set to zero and the rest is stored as a
// block-sparse matrix, which the field kernel then streams instead of the
// dense operator.
//
// Selection.  The cut is an order statistic of the float32 magnitudes above
// 1e-14 of all 9 entries of every block; a SYM6 block stores 6 of them, so
// the off-diagonal components count twice.  Magnitudes of positive floats order
// like their bit patterns, so the cut is found by a three-pass radix select
// over the bit patterns (digits of bits 30..20, 19..9, 8..0): each pass is a
// weighted histogram of the entries that match the digits chosen so far, and
// the host walks the 2048 bins to the one holding rank r.  The result is the
// exact bit pattern of the r-th smallest magnitude.
//
// Structure.  One wave per target tile counts the kept blocks of its row
// (self block, or any component above the cut), the host scans the counts
// into row pointers, and a second pass writes the column indices and the
// component planes, zeroing removed entries.  Kept blocks stay in ascending
// source order, so the structure is unique.  On a single layer of tiles (one
// z for every centre) the xz and yz components of every block are zero (the
// tensor of a tile at a point of its own mid-plane is even in z), so only the
// planes xx, xy, yy, zz are stored: 20 instead of 28 bytes per kept block.
//
// Product.  k_field_bsr: one 256-thread workgroup per target tile streams
// that row's column indices and component planes (coalesced, four blocks per
// thread in flight) and gathers the source states (12 bytes each, served from
// cache), then runs the same fused epilogue as the dense kernel.  (A layout
// with per-segment masks of kept blocks and lane-owned columns, which reads
// the states contiguously, measured slower: idle lanes on dropped columns.)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"
#include "epilogue.h"

namespace tmag {
namespace {

constexpr int kBins = 2048;
// Magnitudes at or below 1e-14 (as float32) are zero up to the float64
// assembly's absolute rounding (entries that vanish by symmetry come out as
// ~1e-17 noise or exact zeros depending on evaluation order); they are not
// ranked.  Physical entries on meshes below ~100 um are far larger.
const uint32_t kZeroFloorBits = __builtin_bit_cast(uint32_t, 1e-14f);

__device__ inline uint32_t mag_bits(float v) { return __float_as_uint(v) & 0x7fffffffu; }

// Pass `pass` of the radix select: histogram of digit `pass` over the nonzero
// entries whose higher digits equal `prefix` (weight 2 for off-diagonal
// components).  Grid: (rows blocks, 6 components); each wave walks rows
// a = 4 blockIdx.x + wave, a += 4 gridDim.x, and each workgroup merges its
// LDS histogram into the global one once.
__global__ __launch_bounds__(256) void k_select_hist(const float* __restrict__ T, int64_t n, int64_t ld,
                                                     int64_t plane, int pass, uint32_t prefix, uint32_t floor,
                                                     unsigned long long* __restrict__ hist) {
    __shared__ uint32_t h[kBins];
    for (int i = threadIdx.x; i < kBins; i += 256) h[i] = 0;
    __syncthreads();
    const int comp = blockIdx.y;
    const uint32_t wgt = (comp == 1 || comp == 2 || comp == 4) ? 2u : 1u;
    for (int64_t a = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6); a < n;
         a += static_cast<int64_t>(gridDim.x) * 4) {
        const float* row = T + comp * plane + a * ld;
        for (int64_t b = threadIdx.x & 63; b < n; b += 64) {
            const uint32_t u = mag_bits(row[b]);
            if (u <= floor) continue;  // zero up to the assembly's rounding
            uint32_t digit;
            bool match;
            if (pass == 0) {
                digit = u >> 20;
                match = true;
            } else if (pass == 1) {
                digit = (u >> 9) & 0x7ffu;
                match = (u >> 20) == prefix;
            } else {
                digit = u & 0x1ffu;
                match = (u >> 9) == prefix;
            }
            if (match) atomicAdd(&h[digit], wgt);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kBins; i += 256)
        if (h[i]) atomicAdd(&hist[i], static_cast<unsigned long long>(h[i]));
}

// Kept blocks per target row: the self block, or any component above the cut.
__device__ inline bool keep_block(const float* T, int64_t plane, int64_t off, bool self, uint32_t cut) {
    if (self) return true;
    bool k = false;
#pragma unroll
    for (int c = 0; c < 6; ++c) k = k || mag_bits(T[c * plane + off]) > cut;
    return k;
}

__global__ __launch_bounds__(256) void k_bsr_count(const float* __restrict__ T, int64_t n, int64_t ld,
                                                   int64_t plane, uint32_t cut, int64_t* __restrict__ cnt) {
    const int64_t a = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (a >= n) return;
    const int lane = threadIdx.x & 63;
    int64_t total = 0;
    for (int64_t b0 = 0; b0 < n; b0 += 64) {
        const int64_t b = b0 + lane;
        const bool k = b < n && keep_block(T, plane, a * ld + b, a == b, cut);
        total += __popcll(__ballot(k));
    }
    if (lane == 0) cnt[a] = total;
}

// Source component of stored plane p: six planes (xx, xy, xz, yy, yz, zz),
// or four (xx, xy, yy, zz) for a single layer.
template <int NP>
__device__ __host__ constexpr int plane_comp(int p) {
    return NP == 6 ? p : (p < 2 ? p : 2 * p - 1);
}

template <int NP>
__global__ __launch_bounds__(256) void k_bsr_fill(const float* __restrict__ T, int64_t n, int64_t ld,
                                                  int64_t plane, uint32_t cut,
                                                  const int64_t* __restrict__ row_ptr,
                                                  int32_t* __restrict__ col, float* __restrict__ vals,
                                                  int64_t nnzb) {
    const int64_t a = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (a >= n) return;
    const int lane = threadIdx.x & 63;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int64_t pos = row_ptr[a];
    for (int64_t b0 = 0; b0 < n; b0 += 64) {
        const int64_t b = b0 + lane;
        const int64_t off = a * ld + b;
        const bool self = a == b;
        const bool k = b < n && keep_block(T, plane, off, self, cut);
        const uint64_t mask = __ballot(k);
        if (k) {
            const int64_t q = pos + __popcll(mask & below);
            col[q] = static_cast<int32_t>(b);
#pragma unroll
            for (int c = 0; c < NP; ++c) {
                const float v = T[plane_comp<NP>(c) * plane + off];
                vals[c * nnzb + q] = (self || mag_bits(v) > cut) ? v : 0.0f;
            }
        }
        pos += __popcll(mask);
    }
}

// Field kernel over a BSR6 operator: one workgroup per (target tile, state).
// Each thread takes four of the row's blocks per round (q, q + 256, ...):
// their column indices and the 24 component loads are issued together, then
// the four gathered source states.  UNI: uniform Ms, applied once to the sum
// instead of per source tile.
template <Epi MODE, bool UNI, int NP>
__global__ __launch_bounds__(256) void k_field_bsr(DevProblem P, const int64_t* __restrict__ row_ptr,
                                                   const int32_t* __restrict__ col,
                                                   const float* __restrict__ vals, int64_t nnzb,
                                                   const float* __restrict__ Ms, float ms_uni, const float* X,
                                                   int64_t sx, EpiArgs E) {
    constexpr int NW = 4;
    constexpr int U = 4;
    constexpr bool STEPPING = MODE == Epi::STAGE || MODE == Epi::RK4_FINAL || MODE == Epi::DP_LAST;
    const int s = blockIdx.y;
    const int a = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    rk4_last_stage_control<MODE>(E);
    bool frozen = false;
    if constexpr (STEPPING) frozen = E.h[s] == 0.0;
    if constexpr (MODE == Epi::STAGE || MODE == Epi::RK4_FINAL) {
        if (frozen) return;
    }
    __shared__ float red[NW][3];
    if (!frozen) {
        const float* x = X + s * sx;
        float hx = 0.0f, hy = 0.0f, hz = 0.0f;
        const int64_t q0 = row_ptr[a], q1 = row_ptr[a + 1];
        auto block = [&](int64_t q, int32_t b) {
            const float ms = UNI ? 1.0f : Ms[b];
            const float mx = x[3 * b] * ms, my = x[3 * b + 1] * ms, mz = x[3 * b + 2] * ms;
            const float xx = vals[q], xy = vals[nnzb + q];
            const float xz = NP == 6 ? vals[2 * nnzb + q] : 0.0f, yy = vals[(NP == 6 ? 3 : 2) * nnzb + q];
            const float yz = NP == 6 ? vals[4 * nnzb + q] : 0.0f, zz = vals[(NP - 1) * nnzb + q];
            hx += xx * mx + xy * my + xz * mz;
            hy += xy * mx + yy * my + yz * mz;
            hz += xz * mx + yz * my + zz * mz;
        };
        int64_t q = q0 + threadIdx.x;
        for (; q + (U - 1) * 256 < q1; q += U * 256) {
            int32_t b[U];
#pragma unroll
            for (int u = 0; u < U; ++u) b[u] = col[q + u * 256];
#pragma unroll
            for (int u = 0; u < U; ++u) block(q + u * 256, b[u]);
        }
        for (; q < q1; q += 256) block(q, col[q]);
        if (UNI) {
            hx *= ms_uni;
            hy *= ms_uni;
            hz *= ms_uni;
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            hx += __shfl_xor(hx, off, 64);
            hy += __shfl_xor(hy, off, 64);
            hz += __shfl_xor(hz, off, 64);
        }
        if (lane == 0) {
            red[wave][0] = hx;
            red[wave][1] = hy;
            red[wave][2] = hz;
        }
        __syncthreads();
    }
    if (wave != 0) return;
    double rmax = 0.0, dmax = 0.0;
    if (!frozen && lane == 0) {
        float h[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float v = 0.0f;
#pragma unroll
            for (int w = 0; w < NW; ++w) v += red[w][c];
            h[c] = -v;
        }
        finish_tile<MODE>(P, X, sx, E, s, a, h[0], h[1], h[2], &rmax, &dmax);
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

// r-th smallest (1-based, weighted) magnitude's bit pattern by radix select.
dim3 hist_grid(int64_t n) { return dim3(static_cast<unsigned>(std::min<int64_t>((n + 3) / 4, 256)), 6); }

tm_status select_cut(const Tensor* S, int64_t r, unsigned long long* hist, hipStream_t s, uint32_t* cut) {
    const int64_t n = S->n;
    const dim3 grid = hist_grid(n);
    uint32_t prefix = 0;
    int64_t rank = r;
    std::vector<unsigned long long> h(kBins);
    for (int pass = 0; pass < 3; ++pass) {
        TM_TRY_HIP(hipMemsetAsync(hist, 0, kBins * sizeof(unsigned long long), s));
        k_select_hist<<<grid, 256, 0, s>>>(static_cast<const float*>(S->data), n, S->ld, S->plane, pass,
                                           prefix, kZeroFloorBits, hist);
        TM_TRY_HIP(hipGetLastError());
        TM_TRY_HIP(hipMemcpyAsync(h.data(), hist, kBins * sizeof(unsigned long long),
                                  hipMemcpyDeviceToHost, s));
        TM_TRY_HIP(hipStreamSynchronize(s));
        const int nb = pass == 2 ? 512 : kBins;
        int d = -1;
        for (int i = 0; i < nb; ++i) {
            const int64_t c = static_cast<int64_t>(h[i]);
            if (rank <= c) {
                d = i;
                break;
            }
            rank -= c;
        }
        TM_REQUIRE(d >= 0, TM_EDEVICE, "tm_tensor_threshold: selection lost rank %lld in pass %d",
                   static_cast<long long>(r), pass);
        // prefix = the magnitude's bits above the next digit
        prefix = (prefix << (pass == 0 ? 0 : (pass == 1 ? 11 : 9))) | static_cast<uint32_t>(d);
    }
    *cut = prefix;
    return TM_OK;
}

// Total weighted count of nonzero entries (= the first pass's histogram sum).
tm_status count_nonzero(const Tensor* S, unsigned long long* hist, hipStream_t s, int64_t* K) {
    const int64_t n = S->n;
    const dim3 grid = hist_grid(n);
    TM_TRY_HIP(hipMemsetAsync(hist, 0, kBins * sizeof(unsigned long long), s));
    k_select_hist<<<grid, 256, 0, s>>>(static_cast<const float*>(S->data), n, S->ld, S->plane, 0, 0u,
                                       kZeroFloorBits, hist);
    TM_TRY_HIP(hipGetLastError());
    std::vector<unsigned long long> h(kBins);
    TM_TRY_HIP(hipMemcpyAsync(h.data(), hist, kBins * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    TM_TRY_HIP(hipStreamSynchronize(s));
    int64_t k = 0;
    for (unsigned long long v : h) k += static_cast<int64_t>(v);
    *K = k;
    return TM_OK;
}

template <Epi MODE, int NP>
void launch_bsr_np(const DevProblem& P, const Tensor* T, const float* Ms, bool uni, float ms_uni, int64_t B,
                   const float* X, int64_t sx, const EpiArgs& e, hipStream_t s) {
    const dim3 grid(static_cast<unsigned>(T->n), static_cast<unsigned>(B));
    if (uni)
        launch_op(k_field_bsr<MODE, true, NP>, grid, dim3(256), s, P, T->row_ptr, T->col,
                  static_cast<const float*>(T->data), T->nnzb, Ms, ms_uni, X, sx, e);
    else
        launch_op(k_field_bsr<MODE, false, NP>, grid, dim3(256), s, P, T->row_ptr, T->col,
                  static_cast<const float*>(T->data), T->nnzb, Ms, ms_uni, X, sx, e);
}

template <Epi MODE>
void launch_bsr_t(const DevProblem& P, const Tensor* T, const float* Ms, bool uni, float ms_uni, int64_t B,
                  const float* X, int64_t sx, const EpiArgs& e, hipStream_t s) {
    if (T->bsr_planes == 4)
        launch_bsr_np<MODE, 4>(P, T, Ms, uni, ms_uni, B, X, sx, e, s);
    else
        launch_bsr_np<MODE, 6>(P, T, Ms, uni, ms_uni, B, X, sx, e, s);
}

}  // namespace

tm_status launch_field_bsr(const Problem* p, Epi mode, int64_t B, const float* X, const EpiArgs& e,
                           hipStream_t s) {
    const Tensor* T = p->T;
    TM_REQUIRE(T->layout == TM_LAYOUT_BSR6 && T->row_ptr && T->col && T->data, TM_EINVAL,
               "sparse field evaluation needs a BSR6 operator");
    TM_REQUIRE(B >= 1 && B <= 65535, TM_EINVAL, "sparse field evaluation: %lld states",
               static_cast<long long>(B));
    const DevProblem P = p->dev();
    const int64_t sx = 3 * p->np;
    const bool uni = p->uniform_ms;
    const float msu = static_cast<float>(p->ms_ref);
    switch (mode) {
        case Epi::HD: launch_bsr_t<Epi::HD>(P, T, p->Ms, uni, msu, B, X, sx, e, s); break;
        case Epi::HEFF: launch_bsr_t<Epi::HEFF>(P, T, p->Ms, uni, msu, B, X, sx, e, s); break;
        case Epi::DMDT: launch_bsr_t<Epi::DMDT>(P, T, p->Ms, uni, msu, B, X, sx, e, s); break;
        case Epi::STAGE: launch_bsr_t<Epi::STAGE>(P, T, p->Ms, uni, msu, B, X, sx, e, s); break;
        case Epi::RK4_FINAL: launch_bsr_t<Epi::RK4_FINAL>(P, T, p->Ms, uni, msu, B, X, sx, e, s); break;
        case Epi::DP_LAST: launch_bsr_t<Epi::DP_LAST>(P, T, p->Ms, uni, msu, B, X, sx, e, s); break;
    }
    TM_TRY_HIP(hipGetLastError());
    return TM_OK;
}

tm_status bsr_rows(const Tensor* T, int64_t a0, int64_t count, double* out) {
    const int64_t n = T->n;
    std::vector<int64_t> rp(count + 1);
    TM_TRY_HIP(hipMemcpy(rp.data(), T->row_ptr + a0, (count + 1) * sizeof(int64_t), hipMemcpyDeviceToHost));
    const int64_t q0 = rp[0], m = rp[count] - rp[0];
    std::vector<int32_t> cols(m);
    std::vector<float> v(6 * m, 0.0f);  // six component planes (xz, yz zero when not stored)
    if (m > 0) {
        TM_TRY_HIP(hipMemcpy(cols.data(), T->col + q0, m * sizeof(int32_t), hipMemcpyDeviceToHost));
        for (int c = 0; c < T->bsr_planes; ++c) {
            const int comp = T->bsr_planes == 6 ? c : plane_comp<4>(c);
            TM_TRY_HIP(hipMemcpy(v.data() + comp * m, static_cast<const float*>(T->data) + c * T->nnzb + q0,
                                 m * sizeof(float), hipMemcpyDeviceToHost));
        }
    }
    std::fill(out, out + count * n * 9, 0.0);
    static const int comp[9] = {0, 1, 2, 1, 3, 4, 2, 4, 5};
    for (int64_t r = 0; r < count; ++r)
        for (int64_t q = rp[r] - q0; q < rp[r + 1] - q0; ++q)
            for (int k = 0; k < 9; ++k) out[(r * n + cols[q]) * 9 + k] = v[comp[k] * m + q];
    return TM_OK;
}

}  // namespace tmag

using namespace tmag;

extern "C" tm_status tm_tensor_threshold(tm_ctx* c, const tm_tensor* src, double frac, hipStream_t stream,
                                         tm_tensor** out) {
    TM_REQUIRE(c && src && out, TM_EINVAL, "tm_tensor_threshold: null argument");
    TM_REQUIRE(src->layout == TM_LAYOUT_SYM6 && src->prec == TM_PREC_FP32 && src->data, TM_EINVAL,
               "tm_tensor_threshold: the source must be an FP32 SYM6 operator");
    TM_REQUIRE(std::isfinite(frac) && frac >= 0.0 && frac <= 1.0, TM_EINVAL,
               "tm_tensor_threshold: fraction %g outside [0, 1]", frac);
    TM_REQUIRE(src->n <= 0x7fffffff, TM_EINVAL, "tm_tensor_threshold: too many tiles");
    TM_TRY_HIP(hipSetDevice(c->device));
    std::unique_lock<std::mutex> lk(c->mu);
    for (auto it = c->cache.begin(); it != c->cache.end(); ++it) {
        Tensor* T = *it;
        if (T->layout == TM_LAYOUT_BSR6 && T->hash == src->hash && T->n == src->n && T->frac == frac &&
            T->centers == src->centers && T->sizes == src->sizes) {
            T->refs += 1;
            c->cache.splice(c->cache.begin(), c->cache, it);
            c->cache_hits += 1;
            *out = static_cast<tm_tensor*>(T);
            return TM_OK;
        }
    }
    c->cache_misses += 1;
    const int64_t n = src->n;
    // scratch: histogram and per-row counts
    const int64_t scratch = kBins * 8 + (n + 1) * 8;
    tm_status st = admit_bytes(c, scratch);
    if (st != TM_OK) return st;
    unsigned long long* hist = nullptr;
    int64_t* cnt = nullptr;
    auto drop_scratch = [&]() {
        if (hist) (void)hipFree(hist);
        if (cnt) (void)hipFree(cnt);
        release_bytes(c, scratch);
    };
    if (hipMalloc(&hist, kBins * 8) != hipSuccess || hipMalloc(&cnt, (n + 1) * 8) != hipSuccess) {
        drop_scratch();
        set_error("tm_tensor_threshold: scratch allocation failed");
        return TM_ENOMEM;
    }
    int64_t K = 0;
    st = count_nonzero(src, hist, stream, &K);
    // rank of the cut among the K nonzero magnitudes (same expression as the
    // definition: r = ceil(frac K), at most K)
    int64_t r = static_cast<int64_t>(std::ceil(frac * static_cast<double>(K)));
    if (r > K) r = K;
    uint32_t cut = 0;  // entries with magnitude bits <= cut are removed (0: only zeros)
    if (st == TM_OK && r > 0) st = select_cut(src, r, hist, stream, &cut);
    const unsigned rgrid = static_cast<unsigned>((n + 3) / 4);
    std::vector<int64_t> rp(n + 1, 0);
    if (st == TM_OK) {
        k_bsr_count<<<rgrid, 256, 0, stream>>>(static_cast<const float*>(src->data), n, src->ld, src->plane, cut,
                                               cnt);
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(rp.data() + 1, cnt, n * 8, hipMemcpyDeviceToHost, stream) != hipSuccess ||
            hipStreamSynchronize(stream) != hipSuccess) {
            set_error("tm_tensor_threshold: block count failed");
            st = TM_EDEVICE;
        }
    }
    if (st != TM_OK) {
        drop_scratch();
        return st;
    }
    for (int64_t a = 0; a < n; ++a) rp[a + 1] += rp[a];
    const int64_t nnzb = rp[n];
    tm_tensor* T = new tm_tensor();
    T->ctx = c;
    T->hash = src->hash;
    T->n = n;
    T->centers = src->centers;
    T->sizes = src->sizes;
    T->prec = TM_PREC_FP32;
    T->layout = TM_LAYOUT_BSR6;
    T->nnzb = nnzb;
    T->frac = frac;
    T->cut = r > 0 ? static_cast<double>(__builtin_bit_cast(float, cut)) : -1.0;
    bool layer = true;  // one z for every centre: xz = yz = 0 in every block
    for (int64_t a = 1; a < n && layer; ++a) layer = src->centers[3 * a + 2] == src->centers[2];
    T->bsr_planes = layer ? 4 : 6;
    T->bytes = 8 * (n + 1) + (4 + 4 * T->bsr_planes) * nnzb;
    st = admit_bytes(c, T->bytes);
    if (st != TM_OK) {
        delete T;
        drop_scratch();
        return st;
    }
    auto fail = [&](tm_status code) {
        release_bytes(c, T->bytes);
        free_tensor(T);
        drop_scratch();
        return code;
    };
    if (hipMalloc(&T->row_ptr, (n + 1) * 8) != hipSuccess ||
        hipMalloc(&T->col, std::max<int64_t>(nnzb, 1) * 4) != hipSuccess ||
        hipMalloc(&T->data, std::max<int64_t>(nnzb, 1) * 4 * T->bsr_planes) != hipSuccess) {
        set_error("tm_tensor_threshold: allocation of %lld blocks failed", static_cast<long long>(nnzb));
        return fail(TM_ENOMEM);
    }
    if (hipMemcpyAsync(T->row_ptr, rp.data(), (n + 1) * 8, hipMemcpyHostToDevice, stream) != hipSuccess)
        return fail(TM_EDEVICE);
    if (T->bsr_planes == 4)
        k_bsr_fill<4><<<rgrid, 256, 0, stream>>>(static_cast<const float*>(src->data), n, src->ld, src->plane, cut,
                                                 T->row_ptr, T->col, static_cast<float*>(T->data), nnzb);
    else
        k_bsr_fill<6><<<rgrid, 256, 0, stream>>>(static_cast<const float*>(src->data), n, src->ld, src->plane, cut,
                                                 T->row_ptr, T->col, static_cast<float*>(T->data), nnzb);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(stream) != hipSuccess) {
        set_error("tm_tensor_threshold: structure fill failed");
        return fail(TM_EDEVICE);
    }
    drop_scratch();
    T->refs = 1;
    c->cache.push_front(T);
    *out = T;
    return TM_OK;
}

extern "C" tm_status tm_tensor_sparse_info(const tm_tensor* t, int64_t* nnzb, double* cut) {
    TM_REQUIRE(t, TM_EINVAL, "tm_tensor_sparse_info: null tensor");
    TM_REQUIRE(t->layout == TM_LAYOUT_BSR6, TM_EINVAL, "tm_tensor_sparse_info: not a BSR6 operator");
    if (nnzb) *nnzb = t->nnzb;
    if (cut) *cut = t->cut;
    return TM_OK;
}

extern "C" tm_status tm_tensor_sparse_get(const tm_tensor* t, int64_t* row_ptr, int32_t* col, float* vals) {
    TM_REQUIRE(t && row_ptr && col && vals, TM_EINVAL, "tm_tensor_sparse_get: null argument");
    TM_REQUIRE(t->layout == TM_LAYOUT_BSR6, TM_EINVAL, "tm_tensor_sparse_get: not a BSR6 operator");
    TM_TRY_HIP(hipSetDevice(t->ctx->device));
    TM_TRY_HIP(hipMemcpy(row_ptr, t->row_ptr, (t->n + 1) * 8, hipMemcpyDeviceToHost));
    if (t->nnzb > 0) {
        TM_TRY_HIP(hipMemcpy(col, t->col, t->nnzb * 4, hipMemcpyDeviceToHost));
        if (t->bsr_planes == 4) std::fill(vals, vals + 6 * t->nnzb, 0.0f);  // xz, yz not stored: zero
        for (int c = 0; c < t->bsr_planes; ++c) {
            const int comp = t->bsr_planes == 6 ? c : plane_comp<4>(c);
            TM_TRY_HIP(hipMemcpy(vals + comp * t->nnzb, static_cast<const float*>(t->data) + c * t->nnzb,
                                 t->nnzb * 4, hipMemcpyDeviceToHost));
        }
    }
    return TM_OK;
}
