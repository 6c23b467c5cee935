// Tensor assembly on the device (float64 arithmetic), and conversion of the
// assembled operator to split bf16 / fp16 storage.
//
// Block (a, b) of the operator is the demagnetisation tensor of cuboid tile b
// evaluated at the centre of tile a (paper Sec. 3: the analytical field of
// each uniformly magnetised tile at the other tiles' centres; the total field
// is the superposition).  With the source box [x1,x2]x[y1,y2]x[z1,z2],
// U_i = x - x_i, V_j = y - y_j, W_k = z - z_k (i = 1 the lower face),
// R_ijk = |(U_i, V_j, W_k)| and corner sign s_i s_j s_k (s_1 = 1, s_2 = -1):
//   N_xx = (1/4pi) sum s_i s_j s_k atan(V_j W_k / (U_i R_ijk))   (cyclic for yy, zz)
//   N_xy = -(1/4pi) sum_ij s_i s_j ln[(W_1 + R_ij1) / (W_2 + R_ij2)]  (xz, yz alike)
// so that the tile's field is H = -N M.  The eight corner radii are shared by
// all six components.  Logarithm ratios are evaluated without cancellation
// (distant tiles would otherwise lose every digit), and an atan term whose
// denominator coordinate is exactly zero is dropped (its four terms cancel).
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include <cmath>

#include "common.h"

namespace tmag {
namespace {

constexpr double kInv4Pi = 1.0 / (4.0 * 3.14159265358979323846);

// ln[(w1 + R1)/(w2 + R2)] with w1 > w2, R_k = sqrt(rho2 + w_k^2).
__device__ inline double log_ratio_dev(double rho2, double w1, double w2, double R1, double R2) {
    const double e = w1 - w2;
    if (w2 >= 0.0) return log1p(e * (1.0 + (w1 + w2) / (R1 + R2)) / (w2 + R2));
    if (w1 <= 0.0) return log1p(e * (1.0 - (w1 + w2) / (R1 + R2)) / (R1 - w1));
    return log((w1 + R1) * (R2 - w2) / rho2);
}

__device__ inline double atan_term(double num, double den) {
    return den == 0.0 ? 0.0 : atan(num / den);
}

// Six components (xx, xy, xz, yy, yz, zz) of the tensor of a box with
// half-edges h at displacement d = (target - box centre).
__device__ void cuboid_tensor(double dx, double dy, double dz, double hx, double hy, double hz,
                              double out[6]) {
    const double U[2] = {dx + hx, dx - hx};
    const double V[2] = {dy + hy, dy - hy};
    const double W[2] = {dz + hz, dz - hz};
    double R[2][2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int k = 0; k < 2; ++k) R[i][j][k] = sqrt(U[i] * U[i] + V[j] * V[j] + W[k] * W[k]);

    double sxx = 0.0, syy = 0.0, szz = 0.0;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const double r = R[i][j][k];
                const double t_xx = atan_term(V[j] * W[k], U[i] * r);
                const double t_yy = atan_term(W[k] * U[i], V[j] * r);
                const double t_zz = atan_term(U[i] * V[j], W[k] * r);
                if ((i + j + k) & 1) {
                    sxx -= t_xx; syy -= t_yy; szz -= t_zz;
                } else {
                    sxx += t_xx; syy += t_yy; szz += t_zz;
                }
            }
    double sxy = 0.0, sxz = 0.0, syz = 0.0;
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const double sg = ((p + q) & 1) ? -1.0 : 1.0;
            // xy: logs in W over the (U_p, V_q) columns
            sxy += sg * log_ratio_dev(U[p] * U[p] + V[q] * V[q], W[0], W[1], R[p][q][0], R[p][q][1]);
            // xz: logs in V over the (U_p, W_q) columns
            sxz += sg * log_ratio_dev(U[p] * U[p] + W[q] * W[q], V[0], V[1], R[p][0][q], R[p][1][q]);
            // yz: logs in U over the (V_p, W_q) columns
            syz += sg * log_ratio_dev(V[p] * V[p] + W[q] * W[q], U[0], U[1], R[0][p][q], R[1][p][q]);
        }
    out[0] = kInv4Pi * sxx;
    out[1] = -kInv4Pi * sxy;
    out[2] = -kInv4Pi * sxz;
    out[3] = kInv4Pi * syy;
    out[4] = -kInv4Pi * syz;
    out[5] = kInv4Pi * szz;
}

template <typename OutT>
__device__ inline OutT cvt(double v);
template <>
__device__ inline float cvt<float>(double v) { return static_cast<float>(v); }
template <>
__device__ inline double cvt<double>(double v) { return v; }

// One thread per (target a, source b); columns b >= n are zero padding.
// SYM6: out[c * plane + a * ld + b].
template <typename OutT>
__global__ __launch_bounds__(256) void k_assemble_sym6(int32_t n, int64_t ld, int64_t plane,
                                                       const double* __restrict__ centers,
                                                       const double* __restrict__ sizes,
                                                       OutT* __restrict__ out) {
    const int64_t b = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t a = blockIdx.y;
    if (b >= ld) return;
    double t6[6] = {0, 0, 0, 0, 0, 0};
    if (b < n) {
        const double dx = centers[3 * a + 0] - centers[3 * b + 0];
        const double dy = centers[3 * a + 1] - centers[3 * b + 1];
        const double dz = centers[3 * a + 2] - centers[3 * b + 2];
        cuboid_tensor(dx, dy, dz, 0.5 * sizes[3 * b + 0], 0.5 * sizes[3 * b + 1],
                      0.5 * sizes[3 * b + 2], t6);
    }
    OutT* p = out + a * ld + b;
#pragma unroll
    for (int c = 0; c < 6; ++c) p[c * plane] = cvt<OutT>(t6[c]);
}

// DENSE9: out[(3a+i) * ld + 3b + j]; rows [3n, rows) and columns [3n, ld)
// are zeroed by the host beforehand.
template <typename OutT>
__global__ __launch_bounds__(256) void k_assemble_dense9(int32_t n, int64_t ld,
                                                         const double* __restrict__ centers,
                                                         const double* __restrict__ sizes,
                                                         OutT* __restrict__ out) {
    const int64_t b = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t a = blockIdx.y;
    if (b >= n) return;
    double t6[6];
    const double dx = centers[3 * a + 0] - centers[3 * b + 0];
    const double dy = centers[3 * a + 1] - centers[3 * b + 1];
    const double dz = centers[3 * a + 2] - centers[3 * b + 2];
    cuboid_tensor(dx, dy, dz, 0.5 * sizes[3 * b + 0], 0.5 * sizes[3 * b + 1], 0.5 * sizes[3 * b + 2],
                  t6);
    OutT* r0 = out + (3 * a) * ld + 3 * b;
    OutT* r1 = r0 + ld;
    OutT* r2 = r1 + ld;
    r0[0] = cvt<OutT>(t6[0]); r0[1] = cvt<OutT>(t6[1]); r0[2] = cvt<OutT>(t6[2]);
    r1[0] = cvt<OutT>(t6[1]); r1[1] = cvt<OutT>(t6[3]); r1[2] = cvt<OutT>(t6[4]);
    r2[0] = cvt<OutT>(t6[2]); r2[1] = cvt<OutT>(t6[4]); r2[2] = cvt<OutT>(t6[5]);
}

// Stored place of tile-order element (r, k) of a blocked DENSE9 operator
// (-1: a zero block of the component-blocked form, not stored).
__device__ inline int64_t store_index(bool cblk, int64_t ld, int vec, int64_t r, int64_t k) {
    return cblk ? dense9c_index(ld / 3, vec, r, k) : dense9_index(ld, vec, r, k);
}

// Split float32 entries (row-major src, rows x ld) into bf16 hi + lo (hi + lo
// carries 16 significant bits), written in the blocked product order.
__global__ __launch_bounds__(256) void k_split_bf16(int64_t rows, int64_t ld, bool cblk, const float* __restrict__ src,
                                                    __hip_bfloat16* __restrict__ hi,
                                                    __hip_bfloat16* __restrict__ lo) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= rows * ld) return;
    const int64_t o = store_index(cblk, ld, 8, i / ld, i % ld);
    if (o < 0) return;
    const float v = src[i];
    const __hip_bfloat16 h = __float2bfloat16(v);
    hi[o] = h;
    lo[o] = __float2bfloat16(v - __bfloat162float(h));
}

// Row-major float32 (rows x ld) to the blocked product order.
__global__ __launch_bounds__(256) void k_block_fp32(int64_t rows, int64_t ld, bool cblk, const float* __restrict__ src,
                                                    float* __restrict__ dst) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= rows * ld) return;
    const int64_t o = store_index(cblk, ld, 4, i / ld, i % ld);
    if (o >= 0) dst[o] = src[i];
}

// Per-row power-of-two scale so that the row maximum maps to [2^13, 2^14),
// then fp16 hi + lo of the scaled row in the blocked product order.  One
// block per row.
__global__ __launch_bounds__(256) void k_split_fp16_rows(int64_t ld, bool cblk, const float* __restrict__ src,
                                                         __half* __restrict__ hi,
                                                         __half* __restrict__ lo,
                                                         float* __restrict__ rscale) {
    __shared__ float red[256];
    const int64_t row = blockIdx.x;
    const float* r = src + row * ld;
    float mx = 0.0f;
    for (int64_t c = threadIdx.x; c < ld; c += blockDim.x) mx = fmaxf(mx, fabsf(r[c]));
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    mx = red[0];
    int e = 0;
    if (mx > 0.0f) frexpf(mx, &e);  // mx = f * 2^e, f in [0.5, 1)
    const int sh = 14 - e;          // mx * 2^sh in [2^13, 2^14)
    const float scale = ldexpf(1.0f, sh);
    // the scale belongs to the product's row: component order in the
    // component-blocked form
    if (threadIdx.x == 0) rscale[cblk ? (row % 3) * (ld / 3) + row / 3 : row] = ldexpf(1.0f, -sh);
    for (int64_t c = threadIdx.x; c < ld; c += blockDim.x) {
        const int64_t o = store_index(cblk, ld, 8, row, c);
        if (o < 0) continue;
        const float v = r[c] * scale;
        const __half h = __float2half(v);
        hi[o] = h;
        lo[o] = __float2half(v - __half2float(h));
    }
}

// PSYM6: tile pair p = (I, J), I <= J, holds block (al, bl) = tensor of tile
// kPsTile J + bl at the centre of tile kPsTile I + al as planes [6][kPsTile][kPsTile]; blocks that
// involve a padding index (>= n) are zero.  PSYM4 (NP = 4) keeps the planes
// xx, xy, yy, zz: the xz and yz components are odd in the z offset, which is
// zero for every pair of a single layer.
template <int NP>
__global__ __launch_bounds__(256) void k_assemble_psym(int32_t n, const int32_t* __restrict__ pairs,
                                                       const double* __restrict__ centers,
                                                       const double* __restrict__ sizes,
                                                       float* __restrict__ out) {
    constexpr int TB = kPsTile * kPsTile;
    static_assert(NP == 6 || NP == 4, "six or four planes");
    const int64_t p = blockIdx.x;
    const int64_t I = pairs[2 * p], J = pairs[2 * p + 1];
    float* tile = out + p * NP * TB;
    for (int e = threadIdx.x + 256 * blockIdx.y; e < TB; e += 256 * gridDim.y) {
        const int64_t a = kPsTile * I + e / kPsTile, b = kPsTile * J + e % kPsTile;
        double t6[6] = {0, 0, 0, 0, 0, 0};
        if (a < n && b < n) {
            const double dx = centers[3 * a + 0] - centers[3 * b + 0];
            const double dy = centers[3 * a + 1] - centers[3 * b + 1];
            const double dz = centers[3 * a + 2] - centers[3 * b + 2];
            cuboid_tensor(dx, dy, dz, 0.5 * sizes[3 * b + 0], 0.5 * sizes[3 * b + 1],
                          0.5 * sizes[3 * b + 2], t6);
        }
        if constexpr (NP == 6) {
#pragma unroll
            for (int c = 0; c < 6; ++c) tile[c * TB + e] = static_cast<float>(t6[c]);
        } else {
            tile[0 * TB + e] = static_cast<float>(t6[0]);
            tile[1 * TB + e] = static_cast<float>(t6[1]);
            tile[2 * TB + e] = static_cast<float>(t6[3]);
            tile[3 * TB + e] = static_cast<float>(t6[5]);
        }
    }
}

}  // namespace

tm_status assemble_psym(Tensor* T, const double* d_centers, const double* d_sizes, hipStream_t s) {
    TM_REQUIRE(is_psym(T->layout) && T->prec == TM_PREC_FP32 && T->pairs, TM_EINVAL,
               "pair-symmetric assembly: bad tensor");
    const dim3 grid(static_cast<unsigned>(T->npairs), 4);
    if (T->layout == TM_LAYOUT_PSYM4)
        k_assemble_psym<4><<<grid, 256, 0, s>>>(static_cast<int32_t>(T->n), T->pairs, d_centers, d_sizes,
                                                static_cast<float*>(T->data));
    else
        k_assemble_psym<6><<<grid, 256, 0, s>>>(static_cast<int32_t>(T->n), T->pairs, d_centers, d_sizes,
                                                static_cast<float*>(T->data));
    TM_TRY_HIP(hipGetLastError());
    return TM_OK;
}

namespace {

// Rows [r0, r0 + nrow) of a blocked DENSE9 array back in row-major order.
template <typename E>
__global__ __launch_bounds__(256) void k_gather_dense9(int64_t ld, bool cblk, int vec, int64_t r0, int64_t nrow,
                                                       const E* __restrict__ src, E* __restrict__ dst) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= nrow * ld) return;
    const int64_t o = store_index(cblk, ld, vec, r0 + i / ld, i % ld);
    dst[i] = o >= 0 ? src[o] : E(0);
}

}  // namespace

tm_status dense9_rows_rowmajor(const Tensor* T, const void* src, int64_t r0, int64_t nrow, void* host) {
    TM_REQUIRE(T->layout == TM_LAYOUT_DENSE9 && T->prec != TM_PREC_FP64 && r0 >= 0 && nrow >= 0 &&
                   r0 + nrow <= T->rows,
               TM_EINVAL, "dense9 read-back: rows out of range");
    if (nrow == 0) return TM_OK;
    const int esz = T->prec == TM_PREC_FP32 ? 4 : 2;
    const int vec = T->prec == TM_PREC_FP32 ? 4 : 8;
    const int64_t count = nrow * T->ld;
    void* d = nullptr;
    TM_TRY_HIP(hipMalloc(&d, count * esz));
    const unsigned g = static_cast<unsigned>((count + 255) / 256);
    if (esz == 4)
        k_gather_dense9<float><<<g, 256>>>(T->ld, T->cblk, vec, r0, nrow, static_cast<const float*>(src),
                                           static_cast<float*>(d));
    else
        k_gather_dense9<uint16_t><<<g, 256>>>(T->ld, T->cblk, vec, r0, nrow, static_cast<const uint16_t*>(src),
                                              static_cast<uint16_t*>(d));
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpy(host, d, count * esz, hipMemcpyDeviceToHost);
    (void)hipFree(d);
    if (e != hipSuccess) {
        set_error("dense9 read-back: %s", hipGetErrorString(e));
        return TM_EDEVICE;
    }
    return TM_OK;
}

tm_status assemble_device(Tensor* T, const double* d_centers, const double* d_sizes,
                          hipStream_t s) {
    const int32_t n = static_cast<int32_t>(T->n);
    const dim3 block(256);
    if (is_psym(T->layout)) return assemble_psym(T, d_centers, d_sizes, s);
    if (T->layout == TM_LAYOUT_SYM6) {
        const dim3 grid(static_cast<unsigned>((T->ld + 255) / 256), static_cast<unsigned>(n));
        if (T->prec == TM_PREC_FP32)
            k_assemble_sym6<float><<<grid, block, 0, s>>>(n, T->ld, T->plane, d_centers, d_sizes,
                                                         static_cast<float*>(T->data));
        else
            k_assemble_sym6<double><<<grid, block, 0, s>>>(n, T->ld, T->plane, d_centers, d_sizes,
                                                          static_cast<double*>(T->data));
        TM_TRY_HIP(hipGetLastError());
        return TM_OK;
    }
    const dim3 grid(static_cast<unsigned>((n + 255) / 256), static_cast<unsigned>(n));
    const size_t esz = (T->prec == TM_PREC_FP64) ? 8 : 4;
    const int64_t count = T->rows * T->ld;
    void* dst = T->data;
    float* tmp = nullptr;
    if (T->prec != TM_PREC_FP64) {  // assembled row-major, then stored blocked
        TM_TRY_HIP(hipMallocAsync(reinterpret_cast<void**>(&tmp), count * sizeof(float), s));
        dst = tmp;
    }
    TM_TRY_HIP(hipMemsetAsync(dst, 0, count * esz, s));
    if (T->prec == TM_PREC_FP64)
        k_assemble_dense9<double><<<grid, block, 0, s>>>(n, T->ld, d_centers, d_sizes,
                                                        static_cast<double*>(dst));
    else
        k_assemble_dense9<float><<<grid, block, 0, s>>>(n, T->ld, d_centers, d_sizes,
                                                       static_cast<float*>(dst));
    TM_TRY_HIP(hipGetLastError());
    if (T->prec == TM_PREC_FP32) {
        const unsigned g = static_cast<unsigned>((count + 255) / 256);
        k_block_fp32<<<g, block, 0, s>>>(T->rows, T->ld, T->cblk, tmp, static_cast<float*>(T->data));
        TM_TRY_HIP(hipGetLastError());
    } else if (T->prec == TM_PREC_BF16X3) {
        const unsigned g = static_cast<unsigned>((count + 255) / 256);
        k_split_bf16<<<g, block, 0, s>>>(T->rows, T->ld, T->cblk, tmp, static_cast<__hip_bfloat16*>(T->data),
                                         static_cast<__hip_bfloat16*>(T->lo));
        TM_TRY_HIP(hipGetLastError());
    } else if (T->prec == TM_PREC_FP16X3) {
        k_split_fp16_rows<<<static_cast<unsigned>(T->rows), block, 0, s>>>(
            T->ld, T->cblk, tmp, static_cast<__half*>(T->data), static_cast<__half*>(T->lo), T->rscale);
        TM_TRY_HIP(hipGetLastError());
    }
    if (tmp) TM_TRY_HIP(hipFreeAsync(tmp, s));
    return TM_OK;
}

}  // namespace tmag
