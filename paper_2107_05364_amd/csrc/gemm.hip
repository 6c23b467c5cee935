// Batched demag product on the matrix cores: many states that share one
// geometry turn H_d = -N (Ms m) into one GEMM per right-hand-side evaluation
// (paper Sec. 3.1: the demag operator is a dense 3N x 3N matrix applied to
// the 3N-vector m; here to B such vectors at once).
//
//   C[r][s] = sum_k A[r][k] X[s][k],  A = stored operator (DENSE9),
//   X[s][3b+j] = (Ms_b / Ms_ref) m_{s,b,j}, H_d = -Ms_ref C.
//
// Precisions (accumulation always float32):
//   FP32   : v_mfma_f32_16x16x4_f32, A and X in float32;
//   BF16X3 : A = Ah + Al, X = Xh + Xl in bf16; C = Ah Xh + Ah Xl + Al Xh
//            with v_mfma_f32_32x32x16_bf16 (the lo*lo term is below the
//            float32 rounding of the result);
//   FP16X3 : as BF16X3 with fp16 and a power-of-two scale per operator row
//            (the row maximum maps to 2^13..2^14, far entries stay normal);
//            the scale is removed in the GEMM epilogue.
//
// Work split: a workgroup (4 waves) owns 128 operator rows x all states and
// one K range (split-K), or, in the aligned plan of a single layer, one or
// two such segments (gemm_work); each wave owns 32 rows (two 16-row MFMA
// tiles in FP32, one 32-row tile in the split forms).  K advances in chunks
// of 64.  The operator is stored blocked (dense9_index): one workgroup's rows
// of one chunk are a contiguous 16 KB (16-bit halves, each) or 32 KB
// (float32) span, read straight into registers, 1 KB per wave load.  The
// right operand is in the same fragment order, one contiguous span per
// chunk, written by k_prep or, inside an attempt, by the previous stage's
// k_finish; it is staged once per workgroup in LDS (a plain copy: every LDS
// access is a contiguous 1 KB per wave, free of bank conflicts) and reused
// by the four waves.  Partial sums go to part[slot][state][row] and a
// fixed-order elementwise pass adds the slots, finishes the effective field
// and the Runge-Kutta stage per tile.  The summation order depends only on
// the problem size and the work plan, never on the batch.
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include <type_traits>
#include <utility>

#include "common.h"
#include "epilogue.h"

namespace tmag {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));

constexpr int KC = kGemmKC;                          // K chunk
constexpr int kBlockElems = kGemmRows * kGemmKC;     // elements of one operator block

struct GemmArgs {
    int64_t ld;         // K extent (= 3 np)
    int64_t bpad;       // state stride of the partial sums (>= 16 NST)
    const void* Ahi;    // FP32: the operator; split: hi part (blocked)
    const void* Alo;    // split: lo part (blocked)
    const float* rscale;// FP16X3: 1/scale per row
    const void* Xhi;    // right operand, fragment order, [ld / KC][16 NST x KC]
    const void* Xlo;
    float* part;        // [splits][bpad][rows]
    int64_t rows;       // padded operator rows (multiple of 128)
    int64_t kper;       // K elements per split (multiple of KC)
    int64_t np;         // padded tiles (component extent of the component-blocked form)
    int32_t cblk;       // component-blocked single layer (dense9c_index)
    // work items: the first rb2 row blocks take splits_xy K splits, the
    // others (the z rows of the component-blocked form) splits_z
    int64_t rowblocks, rb2, splits_xy, splits_z;
    // aligned plan (component-blocked form, nq > 0): K cut into nq
    // super-ranges, x/y rows in parts of px chunks, z rows in parts of pz =
    // px / 2; an item is one x/y part or two z parts (of consecutive z row
    // blocks) of one super-range, items numbered super-range by super-range
    int64_t nq, px, pz;
};

// Work items in split-major order: the row blocks of split 0, then of split
// 1, ..., first for the row blocks with the full K range, then for the z
// row blocks of the component-blocked form, whose shorter K range needs
// fewer splits of the same length (no workgroup idles).  Consecutive
// workgroups go to the eight XCDs in turn, each with its own L2; workgroup
// bid takes item (bid mod 8) per + bid / 8, so that every XCD works through
// one contiguous run of items and reads the right operand of only one or
// two K ranges (per = items per XCD; the few workgroups past the last item
// do nothing).  Returns false for those.
constexpr int kXcds = 8;
__device__ inline bool gemm_item(const GemmArgs& G, int64_t bid, int64_t* rb, int64_t* sp) {
    const int64_t total = G.rb2 * G.splits_xy + (G.rowblocks - G.rb2) * G.splits_z;
    const int64_t per = (total + kXcds - 1) / kXcds;
    const int64_t item = (bid % kXcds) * per + bid / kXcds;
    if (item >= total) return false;
    const int64_t nxy = G.rb2 * G.splits_xy;
    if (item < nxy) {
        *rb = item % G.rb2;
        *sp = item / G.rb2;
    } else {
        const int64_t z = item - nxy, nz = G.rowblocks - G.rb2;
        *rb = G.rb2 + z % nz;
        *sp = z / nz;
    }
    return true;
}

// K range [k0, k1) of row block rb and the element offset of its first stored
// block: every K for the dense form; for the component-blocked form the x/y
// columns for the x/y rows and the z columns for the z rows.
__device__ inline void row_block_k(const GemmArgs& G, int64_t rb, int64_t* k0, int64_t* k1, int64_t* base) {
    constexpr int64_t BE = kBlockElems;
    if (!G.cblk) {
        *k0 = 0;
        *k1 = G.ld;
        *base = rb * (G.ld / KC) * BE;
        return;
    }
    const int64_t rb2 = 2 * G.np / kGemmRows, kc2 = 2 * G.np / KC;
    if (rb < rb2) {
        *k0 = 0;
        *k1 = 2 * G.np;
        *base = rb * kc2 * BE;
    } else {
        *k0 = 2 * G.np;
        *k1 = 3 * G.np;
        *base = (rb2 * kc2 + (rb - rb2) * (G.np / KC)) * BE;
    }
}

// What a workgroup multiplies: one or two segments of consecutive stored
// blocks and K chunks; chunk c of the item is block blkA + c at K chunk
// kcA + c for c < lenA, else block blkB + (c - lenA) at K chunk kcB +
// (c - lenA).  Each segment is summed into partial-sum slot slotA / slotB of
// its row block rbA / rbB.
struct GemmWork {
    int64_t blkA, kcA, blkB, kcB, rbA, rbB;
    int32_t lenA, len, slotA, slotB;
};

// Work of workgroup bid (false past the last item; XCD order as gemm_item).
__device__ inline bool gemm_work(const GemmArgs& G, int64_t bid, GemmWork* w) {
    if (G.nq == 0) {
        int64_t rb, sp;
        if (!gemm_item(G, bid, &rb, &sp)) return false;
        int64_t kfirst, klast, rbase;
        row_block_k(G, rb, &kfirst, &klast, &rbase);
        const int64_t kb = kfirst + sp * G.kper;
        const int64_t ke = min(kb + G.kper, klast);
        // a split past the row block's K range adds nothing: it writes zero partials
        const int32_t nch = ke > kb ? static_cast<int32_t>((ke - kb) / KC) : 0;
        w->blkA = rbase / kBlockElems + (nch > 0 ? (kb - kfirst) / KC : 0);
        w->kcA = (nch > 0 ? kb : kfirst) / KC;
        w->rbA = rb;
        w->slotA = static_cast<int32_t>(sp);
        w->lenA = w->len = nch;
        w->blkB = w->blkA;
        w->kcB = w->kcA;
        w->rbB = rb;
        w->slotB = w->slotA;
        return true;
    }
    const int64_t zrb = G.rowblocks - G.rb2;
    const int64_t per_q = G.rb2 + zrb / 2;  // items per super-range
    const int64_t total = G.nq * per_q;
    const int64_t per = (total + kXcds - 1) / kXcds;
    const int64_t item = (bid % kXcds) * per + bid / kXcds;
    if (item >= total) return false;
    const int64_t q = item / per_q, r = item % per_q;
    const int64_t kc2 = 2 * G.np / KC, kz = G.np / KC;
    w->slotA = w->slotB = static_cast<int32_t>(q);
    if (r < G.rb2) {
        w->rbA = w->rbB = r;
        w->kcA = w->kcB = q * G.px;
        w->blkA = w->blkB = r * kc2 + q * G.px;
        w->lenA = w->len = static_cast<int32_t>(G.px);
    } else {
        const int64_t z = G.rb2 + 2 * (r - G.rb2);  // first of the item's two z row blocks
        w->rbA = z;
        w->rbB = z + 1;
        w->kcA = w->kcB = kc2 + q * G.pz;
        w->blkA = G.rb2 * kc2 + (z - G.rb2) * kz + q * G.pz;
        w->blkB = w->blkA + kz;
        w->lenA = static_cast<int32_t>(G.pz);
        w->len = static_cast<int32_t>(2 * G.pz);
    }
    return true;
}

// Calls f(integral_constant<int, 0>), ..., f(integral_constant<int, N - 1>) in turn.
template <typename F, int... I>
__device__ inline void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ inline void static_for(F&& f) {
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// The work loop of both products over the item's chunks c = 0 .. len - 1,
// chunk c multiplied from register ring slot c mod R.  Per chunk: the X tile
// of chunk c + 1 and the operator rows of chunk c + R - 1 are requested, the
// products of chunk c run (operator rows from the ring, X from LDS buffer
// c mod 2), the X tile goes to LDS buffer (c + 1) mod 2 (which no wave reads
// any more: all passed the barrier after chunk c - 1), one barrier.  Near
// the end the loads repeat the last chunk instead of branching, so that the
// wait counts stay exact.  The addresses of a chunk come from gemm_work's
// segments by a select, so that the requests run ahead across the segment
// boundary; the loop itself is split there: flush(rb, slot) writes a
// segment's partial sums and clears the accumulators between the two loops
// (segment B enters its loop at ring slot lenA mod R), without a branch per
// chunk and without draining the pipeline.
template <int R, bool SEG2, typename LX, typename LA, typename CP, typename SX, typename FL>
__device__ inline void gemm_run(const GemmWork& W, LX&& load_x, LA&& load_a, CP&& compute, SX&& store_x,
                                FL&& flush) {
    const int last = W.len - 1;
    auto step = [&](auto slot, int c) {
        constexpr int S = decltype(slot)::value;
        load_x(min(c + 1, last));
        load_a(std::integral_constant<int, (S + R - 1) % R>{}, min(c + R - 1, last));
        compute(slot, c & 1);
        store_x((c + 1) & 1);
        __syncthreads();
    };
    // chunks [c0, c1): a head up to the next multiple of R (branches once
    // per segment), then whole rounds of the ring, then the tail
    auto run = [&](int c0, int c1) {
        int c = c0;
        if constexpr (SEG2) {
            static_for<R - 1>([&](auto k) {
                constexpr int S = decltype(k)::value + 1;
                if (c < c1 && c % R == S) {
                    step(std::integral_constant<int, S>{}, c);
                    ++c;
                }
            });
        }
        for (; c + R <= c1; c += R) static_for<R>([&](auto k) { step(k, c + decltype(k)::value); });
        static_for<R - 1>([&](auto k) {
            if (c + decltype(k)::value < c1) step(k, c + decltype(k)::value);
        });
    };
    if (W.len > 0) {
        load_x(0);
        static_for<R - 1>([&](auto k) { load_a(k, min(static_cast<int>(decltype(k)::value), last)); });
        store_x(0);
        __syncthreads();
    }
    if (SEG2 && W.lenA < W.len) {
        run(0, W.lenA);
        flush(W.rbA, W.slotA);
        run(W.lenA, W.len);
        flush(W.rbB, W.slotB);
    } else {
        run(0, W.len);
        flush(W.rbA, W.slotA);
    }
}

template <int PREC>
struct Elt;
template <>
struct Elt<0> { using T = float; using V = float4; static constexpr int kVec = 4; };
template <>
struct Elt<1> { using T = __bf16; using V = v8bf; static constexpr int kVec = 8; };
template <>
struct Elt<2> { using T = _Float16; using V = v8h; static constexpr int kVec = 8; };

typedef float v16f __attribute__((ext_vector_type(16)));

// 32x32x16 products of the split forms: lane l holds A row l % 32 and B
// column l % 32, each at K 8 (l / 32) .. +7; the result element 4 i + j of
// lane l is row 8 i + 4 (l / 32) + j, column l % 32.  (On this part the
// 32x32x16 form runs at about 1.8 times the rate of the 16x16x32 form.)
template <int PREC, typename AV>
__device__ inline v16f mfma_split(const AV& a, const AV& b, const v16f& c) {
    if constexpr (PREC == 1) return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    else return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}

// FP32 product on 16x16x4 MFMAs: a workgroup (4 waves) owns 128 operator
// rows at a time, wave w two 16-row tiles, x all NST 16-state tiles, over
// its work (gemm_work, gemm_run).  One wave per SIMD (the register file
// holds R chunks of operator rows); the MFMAs sweep the independent
// accumulators so that none waits for its predecessor.
template <int PREC, int NST, int R, bool SEG2>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_gemm(GemmArgs G) {
    static_assert(PREC == 0, "the split forms use k_gemm_split");
    using T = typename Elt<PREC>::T;
    using AV = typename Elt<PREC>::V;
    constexpr int VEC = Elt<PREC>::kVec;
    constexpr int NSUB = KC / (4 * VEC);                       // MFMA K steps per chunk
    constexpr int NS = NST * 16;
    constexpr int XB = NS * KC * static_cast<int>(sizeof(T));  // bytes of one X array per chunk
    constexpr int XPIECES = XB / 16;
    constexpr int XPT = (XPIECES + 255) / 256;                 // 16-byte pieces per thread
    __shared__ __attribute__((aligned(16))) unsigned char lds[2 * XB];

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = lane >> 4, j = lane & 15;
    GemmWork W;
    if (!gemm_work(G, blockIdx.x, &W)) return;
    const T* Ah = static_cast<const T*>(G.Ahi);
    const unsigned char* Xh = static_cast<const unsigned char*>(G.Xhi);
    // a plan with one segment per item (SEG2 false) addresses without a select
    auto blk_of = [&](int c) { return !SEG2 || c < W.lenA ? W.blkA + c : W.blkB + (c - W.lenA); };
    auto kc_of = [&](int c) { return !SEG2 || c < W.lenA ? W.kcA + c : W.kcB + (c - W.lenA); };

    v4f acc[2][NST];
    auto zero = [&]() {
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int s = 0; s < NST; ++s) acc[r][s] = v4f{0.f, 0.f, 0.f, 0.f};
    };
    zero();

    v4u xh_r[XPT];
    // operator rows of R chunks: the one being multiplied and the next in flight
    AV ah[R][NSUB][2];

    auto load_x = [&](int c) {
        const int64_t base = kc_of(c) * XB;
#pragma unroll
        for (int q = 0; q < XPT; ++q) {
            const int idx = threadIdx.x + 256 * q;
            if (XPIECES % 256 == 0 || idx < XPIECES) xh_r[q] = *reinterpret_cast<const v4u*>(Xh + base + 16 * idx);
        }
    };
    auto store_x = [&](int buf) {
        unsigned char* base = lds + buf * XB;
#pragma unroll
        for (int q = 0; q < XPT; ++q) {
            const int idx = threadIdx.x + 256 * q;
            if (XPIECES % 256 == 0 || idx < XPIECES) *reinterpret_cast<v4u*>(base + 16 * idx) = xh_r[q];
        }
    };
    // chunk rows go to ring slot S (a compile-time index, so the ring stays in registers)
    auto load_a = [&](auto slot, int c) {
        constexpr int S = decltype(slot)::value;
        const int64_t cb = blk_of(c) * kBlockElems;
#pragma unroll
        for (int sub = 0; sub < NSUB; ++sub)
#pragma unroll
            for (int rt = 0; rt < 2; ++rt) {
                const int64_t off = cb + static_cast<int64_t>(((wave * NSUB + sub) * 2 + rt) * 64 + lane) * VEC;
                ah[S][sub][rt] = *reinterpret_cast<const AV*>(Ah + off);
            }
    };
    auto compute = [&](auto slot, int buf) {
        constexpr int S = decltype(slot)::value;
        const auto& hi = ah[S];
        const unsigned char* xs = lds + buf * XB;
#pragma unroll
        for (int sub = 0; sub < NSUB; ++sub) {
            float4 b[NST];
#pragma unroll
            for (int st = 0; st < NST; ++st)
                b[st] = *reinterpret_cast<const float4*>(xs + ((sub * NST + st) * 64 + lane) * 16);
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
        }
        // the next chunks' global loads (issued above in program order) are
        // spread over the products so that they co-issue with the MFMAs
        constexpr int NMF = NSUB * 4 * NST * 2;    // MFMAs per chunk
        constexpr int NVM = NSUB * 2 + XPT;        // global loads per chunk
#pragma unroll
        for (int i = 0; i < NVM; ++i) {
            __builtin_amdgcn_sched_group_barrier(0x008, NMF / NVM, 0);  // MFMA
            __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);          // VMEM read
        }
    };
    // D[4 g + r][j] of tile (rt, st) -> part[slot][state 16 st + j][row 128 rb + 32 wave + 16 rt + 4 g + r]
    auto flush = [&](int64_t rb, int32_t slot) {
        float* out = G.part + slot * G.bpad * G.rows;
        const int64_t rowbase = rb * kGemmRows + wave * 32;
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) {
            const int64_t r0 = rowbase + 16 * rt + 4 * g;
#pragma unroll
            for (int st = 0; st < NST; ++st) {
                const v4f v = acc[rt][st];
                *reinterpret_cast<float4*>(out + (16 * st + j) * G.rows + r0) = make_float4(v.x, v.y, v.z, v.w);
            }
        }
        zero();
    };
    gemm_run<R, SEG2>(W, load_x, load_a, compute, store_x, flush);
}

// The split forms (BF16X3, FP16X3) on 32x32x16 MFMAs: a workgroup (4 waves)
// owns 128 operator rows at a time, wave w one 32-row tile, x all NSB
// 32-state tiles, over its work (gemm_work, gemm_run).  Per K chunk of 64
// (four K steps of 16) a lane loads its operator row's hi and lo halves for
// each step (16 bytes each, the blocked order: 1 KB per wave load) and the B
// fragments from the LDS copy of the X chunk; per K step three sweeps
// (hi hi, hi lo, lo hi) over the NSB independent accumulators.
template <int PREC, int NSB, int R, bool SEG2>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_gemm_split(GemmArgs G) {
    static_assert(PREC == 1 || PREC == 2, "split forms only");
    using T = typename Elt<PREC>::T;
    using AV = typename Elt<PREC>::V;
    constexpr int KS = KC / 16;                                // K steps per chunk
    constexpr int NS = NSB * 32;
    constexpr int XB = NS * KC * static_cast<int>(sizeof(T));  // bytes of one X array per chunk
    constexpr int XPIECES = XB / 16;
    constexpr int XPT = (XPIECES + 255) / 256;
    constexpr int BUF = 2 * XB;
    __shared__ __attribute__((aligned(16))) unsigned char lds[2 * BUF];

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    GemmWork W;
    if (!gemm_work(G, blockIdx.x, &W)) return;
    const T* Ah = static_cast<const T*>(G.Ahi);
    const T* Al = static_cast<const T*>(G.Alo);
    const unsigned char* Xh = static_cast<const unsigned char*>(G.Xhi);
    const unsigned char* Xl = static_cast<const unsigned char*>(G.Xlo);
    // a plan with one segment per item (SEG2 false) addresses without a select
    auto blk_of = [&](int c) { return !SEG2 || c < W.lenA ? W.blkA + c : W.blkB + (c - W.lenA); };
    auto kc_of = [&](int c) { return !SEG2 || c < W.lenA ? W.kcA + c : W.kcB + (c - W.lenA); };

    v16f acc[NSB];
    auto zero = [&]() {
#pragma unroll
        for (int s = 0; s < NSB; ++s)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[s][e] = 0.0f;
    };
    zero();

    v4u xh_r[XPT], xl_r[XPT];
    AV ah[R][KS], al[R][KS];

    auto load_x = [&](int c) {
        const int64_t base = kc_of(c) * XB;
#pragma unroll
        for (int q = 0; q < XPT; ++q) {
            const int idx = threadIdx.x + 256 * q;
            if (XPIECES % 256 == 0 || idx < XPIECES) {
                const int64_t off = base + 16 * idx;
                xh_r[q] = *reinterpret_cast<const v4u*>(Xh + off);
                xl_r[q] = *reinterpret_cast<const v4u*>(Xl + off);
            }
        }
    };
    auto store_x = [&](int buf) {
        unsigned char* base = lds + buf * BUF;
#pragma unroll
        for (int q = 0; q < XPT; ++q) {
            const int idx = threadIdx.x + 256 * q;
            if (XPIECES % 256 == 0 || idx < XPIECES) {
                *reinterpret_cast<v4u*>(base + 16 * idx) = xh_r[q];
                *reinterpret_cast<v4u*>(base + XB + 16 * idx) = xl_r[q];
            }
        }
    };
    auto load_a = [&](auto slot, int c) {
        constexpr int S = decltype(slot)::value;
        const int64_t cb = blk_of(c) * kBlockElems;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const int64_t off = cb + static_cast<int64_t>((wave * KS + ks) * 64 + lane) * 8;
            ah[S][ks] = *reinterpret_cast<const AV*>(Ah + off);
            al[S][ks] = *reinterpret_cast<const AV*>(Al + off);
        }
    };
    auto compute = [&](auto slot, int buf) {
        constexpr int S = decltype(slot)::value;
        const unsigned char* xs = lds + buf * BUF;
        // the B fragments of two K steps are requested ahead of their products
#pragma unroll
        for (int k2 = 0; k2 < KS; k2 += 2) {
            AV bh[2][NSB], bl[2][NSB];
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int st = 0; st < NSB; ++st) {
                    const int o = (((k2 + u) * NSB + st) * 64 + lane) * 16;
                    bh[u][st] = *reinterpret_cast<const AV*>(xs + o);
                    bl[u][st] = *reinterpret_cast<const AV*>(xs + XB + o);
                }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int ks = k2 + u;
#pragma unroll
                for (int st = 0; st < NSB; ++st) acc[st] = mfma_split<PREC>(ah[S][ks], bh[u][st], acc[st]);
#pragma unroll
                for (int st = 0; st < NSB; ++st) acc[st] = mfma_split<PREC>(ah[S][ks], bl[u][st], acc[st]);
#pragma unroll
                for (int st = 0; st < NSB; ++st) acc[st] = mfma_split<PREC>(al[S][ks], bh[u][st], acc[st]);
            }
        }
        // the next chunks' global loads (issued above in program order) are
        // spread over the products so that they co-issue with the MFMAs
        constexpr int NMF = 3 * KS * NSB;      // MFMAs per chunk
        constexpr int NVM = 2 * KS + 2 * XPT;  // global loads per chunk
#pragma unroll
        for (int i = 0; i < NVM; ++i) {
            __builtin_amdgcn_sched_group_barrier(0x008, NMF / NVM > 0 ? NMF / NVM : 1, 0);  // MFMA
            __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);                            // VMEM read
        }
    };
    // element 4 i + j of tile st -> part[slot][state 32 st + l % 32][row 128 rb + 32 wave + 8 i + 4 (l / 32) + j]
    const int col = lane & 31, h = lane >> 5;
    auto flush = [&](int64_t rb, int32_t slot) {
        float* out = G.part + slot * G.bpad * G.rows;
        const int64_t rowbase = rb * kGemmRows + wave * 32;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t r0 = rowbase + 8 * i + 4 * h;
            float4 sc = make_float4(1.f, 1.f, 1.f, 1.f);
            if constexpr (PREC == 2) sc = *reinterpret_cast<const float4*>(G.rscale + r0);
#pragma unroll
            for (int st = 0; st < NSB; ++st)
                *reinterpret_cast<float4*>(out + (32 * st + col) * G.rows + r0) =
                    make_float4(acc[st][4 * i] * sc.x, acc[st][4 * i + 1] * sc.y, acc[st][4 * i + 2] * sc.z,
                                acc[st][4 * i + 3] * sc.w);
        }
        zero();
    };
    gemm_run<R, SEG2>(W, load_x, load_a, compute, store_x, flush);
}

// Right operand from the (padded) stage input Y [B][ld]: (Ms_b / Ms_ref) m,
// as float32 or split into hi + lo, written in the product's fragment order,
// chunk kc (KC columns of ns states) after chunk kc - 1:
//   float32 (16-state tiles, nt = ns / 16): state 16 st + j, column
//     kc KC + 16 sub + 4 g + e at ((sub nt + st) 64 + 16 g + j) 4 + e;
//   split forms (32-state tiles, nt = ns / 32): state 32 st + i, column
//     kc KC + 16 ks + 8 q + e at ((ks nt + st) 64 + 32 q + i) 8 + e;
// states B .. ns - 1 and tiles n .. np - 1 are zero.  With the
// component-blocked operator, K is in component order as well: column k
// holds component k / np of tile k % np.
// One workgroup per 64 tiles and 16 states: the 16 x 192 stage-input values
// of its tiles (three components each) come in as coalesced 16-byte loads,
// are scaled (Ms from LDS) into an LDS tile, and leave as the 16-byte
// fragment pieces of the three chunks they make (dense form: columns 3 b0 ..
// 3 b0 + 191; the component-blocked form: the chunk of each component), each
// output piece one contiguous store.
constexpr int kPrepTiles = 64;
constexpr int kPrepStates = 16;
constexpr int kPrepCols = 3 * kPrepTiles;
template <int PREC>
__global__ __launch_bounds__(256) void k_prep(int64_t B, int64_t ns, int64_t ld, int32_t n, bool cblk,
                                              const float* __restrict__ Y, const float* __restrict__ Ms,
                                              float inv_ref, void* __restrict__ xh, void* __restrict__ xl) {
    __shared__ float tile[kPrepStates][kPrepCols + 1];
    __shared__ float msl[kPrepTiles];
    const int t = threadIdx.x;
    const int64_t b0 = static_cast<int64_t>(blockIdx.x) * kPrepTiles;
    const int64_t s0 = static_cast<int64_t>(blockIdx.y) * kPrepStates;
    constexpr int F4 = kPrepCols / 4;  // 16-byte pieces per state row
    constexpr int LR = (kPrepStates * F4 + 255) / 256;
    float4 v[LR];
#pragma unroll
    for (int r = 0; r < LR; ++r) {
        const int f = t + 256 * r, i = f / F4, m = f % F4;
        v[r] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (f < kPrepStates * F4 && s0 + i < B) v[r] = *reinterpret_cast<const float4*>(Y + (s0 + i) * ld + 3 * b0 + 4 * m);
    }
    if (t < kPrepTiles && b0 + t < n) msl[t] = Ms[b0 + t] * inv_ref;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < LR; ++r) {
        const int f = t + 256 * r, i = f / F4, m = f % F4;
        if (f >= kPrepStates * F4) continue;
        const float vv[4] = {v[r].x, v[r].y, v[r].z, v[r].w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int c = 4 * m + e;
            tile[i][c] = b0 + c / 3 < n ? vv[e] * msl[c / 3] : 0.0f;
        }
    }
    __syncthreads();
    const int64_t np = ld / 3;
    const int64_t cs = ns * KC;  // elements of one chunk
    // K chunk and LDS column of chunk-local column kk of output chunk j
    auto chunk = [&](int j) { return cblk ? (j * np + b0) / KC : 3 * b0 / KC + j; };
    auto col = [&](int j, int kk) { return cblk ? 3 * kk + j : KC * j + kk; };
    if constexpr (PREC == 0) {
        // float32: the workgroup's states are 16-state tile st = blockIdx.y; 256 float4 pieces per chunk
        const int64_t nt = ns / 16, st = blockIdx.y;
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const int pc = t + 256 * r, j = pc / 256, w = pc % 256;
            const int sub = w / 64, g = (w % 64) / 16, jj = w % 16, kk = 16 * sub + 4 * g;
            const float4 o = make_float4(tile[jj][col(j, kk)], tile[jj][col(j, kk + 1)], tile[jj][col(j, kk + 2)],
                                         tile[jj][col(j, kk + 3)]);
            *reinterpret_cast<float4*>(static_cast<float*>(xh) + chunk(j) * cs + ((sub * nt + st) * 64 + 16 * g + jj) * 4) = o;
        }
    } else {
        // split forms: the workgroup's states are half h of 32-state tile st; 128 pieces per chunk
        using T = typename Elt<PREC>::T;
        using AV = typename Elt<PREC>::V;
        const int64_t nt = ns / 32, st = blockIdx.y / 2;
        const int h = blockIdx.y % 2;
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int pc = t + 256 * r;
            if (pc >= 3 * 128) break;
            const int j = pc / 128, w = pc % 128;
            const int ks = w / 32, q = (w % 32) / 16, il = w % 16, kk = 16 * ks + 8 * q;
            AV hi, lo;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const float x = tile[il][col(j, kk + e)];
                const T hv = static_cast<T>(x);
                hi[e] = hv;
                lo[e] = static_cast<T>(x - static_cast<float>(hv));
            }
            const int64_t o = chunk(j) * cs + ((ks * nt + st) * 64 + 32 * q + 16 * h + il) * 8;
            *reinterpret_cast<AV*>(static_cast<T*>(xh) + o) = hi;
            *reinterpret_cast<AV*>(static_cast<T*>(xl) + o) = lo;
        }
    }
}

// Where a stage writes the right operand of its output (the next stage's
// input) as well: the fragment arrays, the padded state count and 1 / Ms_ref.
struct FragOut {
    void* xh = nullptr;
    void* xl = nullptr;
    int64_t ns = 0;
    float inv = 0.0f;
};

// Sum of the split-K partials in fixed order, then the per-tile finish.
// Rows are in component order for the component-blocked operator (row
// i np + a holds component i of tile a), else in tile order (3 a + i).
// splits_z: the partials of the z rows of the component-blocked operator
// (= splits in the dense form).  A stage launch with F.xh set also writes
// its output's right operand, the values k_prep would make of it, so that
// the next stage's product needs no k_prep.
template <Epi MODE, int PREC>
__global__ __launch_bounds__(256) void k_finish(DevProblem P, const float* __restrict__ part,
                                                int64_t splits, int64_t splits_z, int64_t bpad, int64_t rows,
                                                bool cblk, float scale, const float* __restrict__ X, int64_t sx,
                                                EpiArgs E, FragOut F) {
    const int s = blockIdx.y;
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    rk4_last_stage_control<MODE>(E);
    double rmax = 0.0, dmax = 0.0;
    float yv[3] = {0.0f, 0.0f, 0.0f};  // the stage output of tile a (STAGE)
    if (a < P.n) {
        const int64_t r0 = cblk ? a : 3 * static_cast<int64_t>(a);
        const int64_t rs = cblk ? P.np : 1;  // row stride between the components
        float h0 = 0.f, h1 = 0.f, h2 = 0.f;
        for (int64_t sp = 0; sp < splits; ++sp) {
            const float* pp = part + (sp * bpad + s) * rows + r0;
            h0 += pp[0];
            h1 += pp[rs];
            if (sp < splits_z) h2 += pp[2 * rs];
        }
        finish_tile<MODE>(P, X, sx, E, s, a, -scale * h0, -scale * h1, -scale * h2, &rmax, &dmax, yv);
    }
    if constexpr (MODE == Epi::STAGE) {
        if (F.xh) {
            // the workgroup's 256 tiles x 3 components of the stage output
            // (the values this thread stored, from registers), scaled, through LDS in
            // column order: component-blocked c 256 + t (column c np + a),
            // dense 3 t + c (column 3 a + c); then whole fragment pieces (8
            // consecutive columns of the split forms, 4 of FP32) leave as
            // 16-byte stores.  Tiles n .. np - 1 are zero, as k_prep makes them.
            __shared__ float fv[3 * 256];
            const int tl = threadIdx.x;
            float v[3] = {0.0f, 0.0f, 0.0f};
            if (a < P.n) {
                const float w = P.Ms[a] * F.inv;
#pragma unroll
                for (int c = 0; c < 3; ++c) v[c] = yv[c] * w;
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) fv[cblk ? c * 256 + tl : 3 * tl + c] = v[c];
            __syncthreads();
            constexpr int VEC = PREC == 0 ? 4 : 8;
            const int64_t a0 = static_cast<int64_t>(blockIdx.x) * 256, np = P.np;
            for (int pc = tl; pc < 3 * 256 / VEC; pc += 256) {
                const int i0 = VEC * pc;
                const int64_t k0 = cblk ? (i0 / 256) * np + a0 + i0 % 256 : 3 * a0 + i0;
                if (cblk ? a0 + i0 % 256 >= np : k0 >= 3 * np) continue;
                const int64_t kc = k0 / KC;
                const int kk = static_cast<int>(k0 % KC);
                if constexpr (PREC == 0) {
                    const int64_t nt = F.ns / 16, st = s / 16;
                    const int j = s % 16, sub = kk / 16, g = (kk % 16) / 4;
                    *reinterpret_cast<float4*>(static_cast<float*>(F.xh) + kc * F.ns * KC +
                                               ((sub * nt + st) * 64 + 16 * g + j) * 4) =
                        make_float4(fv[i0], fv[i0 + 1], fv[i0 + 2], fv[i0 + 3]);
                } else {
                    using T = typename Elt<PREC>::T;
                    using AV = typename Elt<PREC>::V;
                    const int64_t nt = F.ns / 32, st = s / 32;
                    const int i = s % 32, ks = kk / 16, q = (kk % 16) / 8;
                    AV hi, lo;
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const float x = fv[i0 + e];
                        const T hv = static_cast<T>(x);
                        hi[e] = hv;
                        lo[e] = static_cast<T>(x - static_cast<float>(hv));
                    }
                    const int64_t o = kc * F.ns * KC + ((ks * nt + st) * 64 + 32 * q + i) * 8;
                    *reinterpret_cast<AV*>(static_cast<T*>(F.xh) + o) = hi;
                    *reinterpret_cast<AV*>(static_cast<T*>(F.xl) + o) = lo;
                }
            }
        }
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

// workgroups of the 1-D product grid (gemm_work): the items rounded up to a
// whole number per XCD
inline unsigned gemm_items(const GemmArgs& G) {
    const int64_t total = G.nq > 0 ? G.nq * (G.rb2 + (G.rowblocks - G.rb2) / 2)
                                   : G.rb2 * G.splits_xy + (G.rowblocks - G.rb2) * G.splits_z;
    return static_cast<unsigned>((total + kXcds - 1) / kXcds * kXcds);
}

// the aligned plan's items have two segments (SEG2), the split plan's one
template <int PREC, int NST, int R>
void launch_gemm_fp32(const GemmArgs& G, hipStream_t s) {
    if (G.nq) launch_op(k_gemm<PREC, NST, R, true>, dim3(gemm_items(G)), dim3(256), s, G);
    else launch_op(k_gemm<PREC, NST, R, false>, dim3(gemm_items(G)), dim3(256), s, G);
}

template <int PREC, int NSB, int R>
void launch_split_t(const GemmArgs& G, dim3 grid, hipStream_t s) {
    if (G.nq) launch_op(k_gemm_split<PREC, NSB, R, true>, grid, dim3(256), s, G);
    else launch_op(k_gemm_split<PREC, NSB, R, false>, grid, dim3(256), s, G);
}

template <int PREC, int R>
tm_status launch_gemm_split(int nsb, const GemmArgs& G, hipStream_t s) {
    const dim3 grid(gemm_items(G));
    switch (nsb) {
        case 1: launch_split_t<PREC, 1, R>(G, grid, s); break;
        case 2: launch_split_t<PREC, 2, R>(G, grid, s); break;
        case 4: launch_split_t<PREC, 4, R>(G, grid, s); break;
        default:
            set_error("batched product: unsupported 32-state tile count %d", nsb);
            return TM_EINVAL;
    }
    TM_TRY_HIP(hipGetLastError());
    return TM_OK;
}

template <int R>
tm_status launch_gemm_p(int nst, const GemmArgs& G, hipStream_t s) {
    switch (nst) {
        case 1: launch_gemm_fp32<0, 1, R>(G, s); break;
        case 2: launch_gemm_fp32<0, 2, R>(G, s); break;
        case 4: launch_gemm_fp32<0, 4, R>(G, s); break;
        case 8: launch_gemm_fp32<0, 8, R>(G, s); break;
        default:
            set_error("batched product: unsupported state-tile count %d", nst);
            return TM_EINVAL;
    }
    TM_TRY_HIP(hipGetLastError());
    return TM_OK;
}

}  // namespace

int gemm_state_tiles(int64_t B) {
    const int64_t t = (B + 15) / 16;
    return t <= 1 ? 1 : t <= 2 ? 2 : t <= 4 ? 4 : 8;
}

int64_t gemm_state_pad(const Tensor* T, int64_t B) {
    if (T->prec == TM_PREC_FP32) return 16 * gemm_state_tiles(B);
    const int64_t t = (B + 31) / 32;
    return 32 * (t <= 1 ? 1 : t <= 2 ? 2 : 4);
}

int gemm_aligned_nq(const Problem* p, int choice) {
    const Tensor* T = p->T;
    if (choice < kGemmAligned || !T->cblk) return 0;
    const int64_t nq = choice - kGemmAligned, np = T->ld / 3;
    const int64_t kz = np / KC, zrb = T->rows / kGemmRows - 2 * np / kGemmRows;
    // whole parts in every super-range, z row blocks in pairs
    const bool ok = nq >= 2 && nq <= 16 && kz % nq == 0 && zrb % 2 == 0;
    return ok ? static_cast<int>(nq) : 0;
}

int64_t gemm_splits(const Problem* p) {
    // the aligned plan sums one slot per super-range
    if (const int nq = gemm_aligned_nq(p, p->gemm_splits)) return nq;
    const int64_t rowblocks = p->T->rows / kGemmRows;
    const int64_t kchunks = p->T->ld / KC;
    // about one workgroup per CU (one wave per SIMD), unless tuned
    int64_t s = (256 + rowblocks - 1) / rowblocks;
    if (s > 1 && rowblocks * s > 256 + rowblocks / 2) s -= 1;
    if (p->gemm_splits > 0) s = p->gemm_splits;
    return std::max<int64_t>(1, std::min<int64_t>(s, std::min<int64_t>(kchunks, 16)));
}

tm_status launch_field_batched(const Problem* p, Epi mode, int64_t B, const float* X,
                               const EpiArgs& e, hipStream_t s) {
    const Tensor* T = p->T;
    Workspace* w = p->ws.get();
    const int64_t ns = gemm_state_pad(T, B);
    TM_REQUIRE(w && w->part && B <= 128 && w->bpad >= ns, TM_EINVAL,
               "batched product: workspace not prepared for %lld states", static_cast<long long>(B));
    TM_REQUIRE(T->ld % KC == 0 && T->rows % kGemmRows == 0 && T->rows >= T->ld, TM_EINVAL,
               "batched product: operator extent %lld x %lld is not a whole number of blocks",
               static_cast<long long>(T->rows), static_cast<long long>(T->ld));
    TM_REQUIRE(w->xh && (T->prec == TM_PREC_FP32 || w->xl), TM_EINVAL,
               "batched product: workspace has no right-operand buffer");
    const int prec = T->prec == TM_PREC_FP32 ? 0 : T->prec == TM_PREC_BF16X3 ? 1 : 2;
    const int64_t ld = T->ld;
    // stage buffers with a right-operand copy of their own
    auto frag_slot = [&](const float* y) { return y == w->ya ? 0 : y == w->yb ? 1 : y == w->y5 ? 2 : -1; };
    const int fin = frag_slot(X);
    const bool ready = w->frag_chain && fin >= 0 && w->frag_src == X && w->fxh[fin];
    w->frag_chain = false;
    const void* xin_h = ready ? w->fxh[fin] : w->xh;
    const void* xin_l = ready ? w->fxl[fin] : w->xl;
    // right operand, in fragment order, unless the stage that wrote X made it
    if (!ready) {
        TM_REQUIRE(ld % (3 * kPrepTiles) == 0, TM_EINVAL, "batched product: K extent %lld is not whole tile groups",
                   static_cast<long long>(ld));
        const dim3 grid(static_cast<unsigned>(ld / (3 * kPrepTiles)),
                        static_cast<unsigned>((ns + kPrepStates - 1) / kPrepStates));
        const float inv = static_cast<float>(1.0 / p->ms_ref);
        const int32_t n32 = static_cast<int32_t>(p->n);
        if (prec == 0)
            k_prep<0><<<grid, 256, 0, s>>>(B, ns, ld, n32, T->cblk, X, p->Ms, inv, w->xh, nullptr);
        else if (prec == 1)
            k_prep<1><<<grid, 256, 0, s>>>(B, ns, ld, n32, T->cblk, X, p->Ms, inv, w->xh, w->xl);
        else
            k_prep<2><<<grid, 256, 0, s>>>(B, ns, ld, n32, T->cblk, X, p->Ms, inv, w->xh, w->xl);
        TM_TRY_HIP(hipGetLastError());
    }
    GemmArgs G;
    G.ld = ld;
    G.bpad = w->bpad;
    G.Ahi = T->data;
    G.Alo = T->lo;
    G.rscale = T->rscale;
    G.Xhi = xin_h;
    G.Xlo = xin_l;
    G.part = w->part;
    G.rows = T->rows;
    G.np = ld / 3;
    G.cblk = T->cblk ? 1 : 0;
    G.nq = gemm_aligned_nq(p, p->gemm_splits);
    G.px = G.nq ? 2 * G.np / KC / G.nq : 0;
    G.pz = G.px / 2;
    const int64_t splits = gemm_splits(p);
    TM_REQUIRE(splits <= w->part_splits, TM_EINVAL, "batched product: workspace holds %lld K splits, %lld asked",
               static_cast<long long>(w->part_splits), static_cast<long long>(splits));
    // K per split from the longest row K range (all of K, or the x/y columns)
    const int64_t kext = T->cblk ? 2 * G.np : ld;
    G.kper = round_up((kext + splits - 1) / splits, KC);
    const int64_t used_splits = (kext + G.kper - 1) / G.kper;
    const int64_t rowblocks = T->rows / kGemmRows;
    G.rowblocks = rowblocks;
    G.rb2 = T->cblk ? 2 * G.np / kGemmRows : rowblocks;
    G.splits_xy = used_splits;
    G.splits_z = T->cblk ? (G.np + G.kper - 1) / G.kper : used_splits;
    // the finish adds the slots of the plan: nq per row for the aligned one
    const int64_t fin_xy = G.nq ? G.nq : G.splits_xy, fin_z = G.nq ? G.nq : G.splits_z;
    const int nst = static_cast<int>(ns / 16), nsb = static_cast<int>(ns / 32);
    tm_status st = prec == 0 ? launch_gemm_p<3>(nst, G, s) : prec == 1 ? launch_gemm_split<1, 3>(nsb, G, s)
                                                             : launch_gemm_split<2, 3>(nsb, G, s);
    if (st != TM_OK) return st;
    // X holds (Ms_b / Ms_ref) m (or m itself when Ms is uniform): H_d = -Ms_ref C
    const float scale = static_cast<float>(p->ms_ref);
    const DevProblem P = p->dev();
    const dim3 grid(static_cast<unsigned>((p->n + 255) / 256), static_cast<unsigned>(B));
    const int64_t sx = 3 * p->np;
    // a stage whose output is ya, yb or y5 writes that output's right operand too
    FragOut F;
    const int fout = mode == Epi::STAGE ? frag_slot(e.ynext) : -1;
    if (fout >= 0 && w->fxh[fout]) {
        F.xh = w->fxh[fout];
        F.xl = w->fxl[fout];
        F.ns = ns;
        F.inv = static_cast<float>(1.0 / p->ms_ref);
    }
    auto fin_p = [&](auto pc) {
        constexpr int PC = decltype(pc)::value;
        switch (mode) {
            case Epi::HD: k_finish<Epi::HD, PC><<<grid, 256, 0, s>>>(P, w->part, fin_xy, fin_z, w->bpad, T->rows, T->cblk, scale, X, sx, e, F); break;
            case Epi::HEFF: k_finish<Epi::HEFF, PC><<<grid, 256, 0, s>>>(P, w->part, fin_xy, fin_z, w->bpad, T->rows, T->cblk, scale, X, sx, e, F); break;
            case Epi::DMDT: k_finish<Epi::DMDT, PC><<<grid, 256, 0, s>>>(P, w->part, fin_xy, fin_z, w->bpad, T->rows, T->cblk, scale, X, sx, e, F); break;
            case Epi::STAGE: k_finish<Epi::STAGE, PC><<<grid, 256, 0, s>>>(P, w->part, fin_xy, fin_z, w->bpad, T->rows, T->cblk, scale, X, sx, e, F); break;
            case Epi::RK4_FINAL: k_finish<Epi::RK4_FINAL, PC><<<grid, 256, 0, s>>>(P, w->part, fin_xy, fin_z, w->bpad, T->rows, T->cblk, scale, X, sx, e, F); break;
            case Epi::DP_LAST: k_finish<Epi::DP_LAST, PC><<<grid, 256, 0, s>>>(P, w->part, fin_xy, fin_z, w->bpad, T->rows, T->cblk, scale, X, sx, e, F); break;
        }
    };
    if (prec == 0) fin_p(std::integral_constant<int, 0>{});
    else if (prec == 1) fin_p(std::integral_constant<int, 1>{});
    else fin_p(std::integral_constant<int, 2>{});
    w->frag_src = F.xh ? e.ynext : nullptr;
    TM_TRY_HIP(hipGetLastError());
    return TM_OK;
}

}  // namespace tmag
