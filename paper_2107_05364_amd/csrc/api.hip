// C ABI: contexts, geometry, the cached demag operator, problems and the
// single-shot field / right-hand-side / energy calls.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include <hip/hip_fp16.h>

#include "common.h"

namespace tmag {

tm_status assemble_device(Tensor* T, const double* d_centers, const double* d_sizes,
                          hipStream_t s);

namespace {
thread_local std::string g_err;
}

void set_error(const char* fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
}

tm_status admit_bytes(Ctx* c, int64_t bytes) {
    // caller holds c->mu
    if (c->used + bytes <= c->budget) {
        c->used += bytes;
        return TM_OK;
    }
    // evict unreferenced cached tensors, least recently used first
    for (auto it = c->cache.end(); it != c->cache.begin() && c->used + bytes > c->budget;) {
        --it;
        Tensor* T = *it;
        if (T->refs > 0) continue;
        c->used -= T->bytes;
        free_tensor(T);
        it = c->cache.erase(it);
    }
    if (c->used + bytes <= c->budget) {
        c->used += bytes;
        return TM_OK;
    }
    set_error("admission refused: %lld bytes requested, %lld of %lld in use",
              static_cast<long long>(bytes), static_cast<long long>(c->used),
              static_cast<long long>(c->budget));
    return TM_ENOMEM;
}

void release_bytes(Ctx* c, int64_t bytes) { c->used -= bytes; }

void free_tensor(Tensor* T) {
    if (T->data) (void)hipFree(T->data);
    if (T->lo) (void)hipFree(T->lo);
    if (T->rscale) (void)hipFree(T->rscale);
    if (T->row_ptr) (void)hipFree(T->row_ptr);
    if (T->col) (void)hipFree(T->col);
    if (T->pairs) (void)hipFree(T->pairs);
    delete static_cast<tm_tensor*>(T);  // every tensor is created as a tm_tensor
}

Workspace::~Workspace() {
    float* fl[] = {y, ya, yb, y5, k[0], k[1], k[2], k[3], k[4], k[5], k[6], Ha, hd, part};
    for (float* p : fl)
        if (p) (void)hipFree(p);
    void* vp[] = {xh, xl, fxh[0], fxh[1], fxh[2], fxl[0], fxl[1], fxl[2], t, h, dt, t1, h1, steps1, flags1, errp, dmxp, snap, steps, rejected, flags, acc, params, esum, diag, stat, bar,
                  bar_fail};
    for (void* p : vp)
        if (p) (void)hipFree(p);
    if (host_params) (void)hipHostFree(host_params);
    if (host_flags) (void)hipHostFree(host_flags);
    if (host_steps) (void)hipHostFree(host_steps);
    if (host_stat) (void)hipHostFree(host_stat);
    drop_graphs();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
}

void Workspace::drop_graphs() {
    for (hipGraphExec_t* g : {&graph1, &graphP[0], &graphP[1], &graphP[2], &graphK}) {
        if (*g) (void)hipGraphExecDestroy(*g);
        *g = nullptr;
    }
}

}  // namespace tmag

using namespace tmag;

extern "C" {

const char* tm_last_error(void) { return g_err.c_str(); }

int32_t tm_version(void) { return 100; }

tm_status tm_init(int32_t device, tm_ctx** out) {
    TM_REQUIRE(out, TM_EINVAL, "tm_init: out is NULL");
    int count = 0;
    TM_TRY_HIP(hipGetDeviceCount(&count));
    TM_REQUIRE(device >= 0 && device < count, TM_EINVAL, "tm_init: device %d of %d", device, count);
    TM_TRY_HIP(hipSetDevice(device));
    // the fixed scratch of tm_demag_noalloc: its device address, once per device
    tm_status sst = noalloc_setup(device);
    if (sst != TM_OK) return sst;
    size_t fr = 0, tot = 0;
    TM_TRY_HIP(hipMemGetInfo(&fr, &tot));
    tm_ctx* c = new tm_ctx();
    c->device = device;
    const int64_t reserve = int64_t(4) << 30;
    c->budget = static_cast<int64_t>(fr) > reserve ? static_cast<int64_t>(fr) - reserve
                                                    : static_cast<int64_t>(fr) / 2;
    *out = c;
    return TM_OK;
}

tm_status tm_finalize(tm_ctx* c) {
    TM_REQUIRE(c, TM_EINVAL, "tm_finalize: null context");
    {
        std::lock_guard<std::mutex> lk(c->mu);
        TM_REQUIRE(c->live_problems == 0 && c->live_servers == 0, TM_EBUSY,
                   "tm_finalize: %d problems and %d servers still alive", c->live_problems,
                   c->live_servers);
        for (Tensor* T : c->cache) free_tensor(T);
        c->cache.clear();
    }
    delete c;
    return TM_OK;
}

tm_status tm_set_memory_budget(tm_ctx* c, int64_t bytes) {
    TM_REQUIRE(c && bytes > 0, TM_EINVAL, "tm_set_memory_budget: bad arguments");
    std::lock_guard<std::mutex> lk(c->mu);
    c->budget = bytes;
    return TM_OK;
}

tm_status tm_geometry_create(tm_ctx* c, int64_t n, const double* centers, const double* sizes,
                             tm_geom** out) {
    TM_REQUIRE(out && centers && sizes, TM_EINVAL, "tm_geometry_create: null argument");
    TM_REQUIRE(n >= 1 && n < (int64_t(1) << 30), TM_EINVAL, "tm_geometry_create: n = %lld",
               static_cast<long long>(n));
    for (int64_t i = 0; i < 3 * n; ++i) {
        TM_REQUIRE(std::isfinite(centers[i]), TM_EINVAL, "tm_geometry_create: centre %lld not finite",
                   static_cast<long long>(i / 3));
        TM_REQUIRE(std::isfinite(sizes[i]) && sizes[i] > 0.0, TM_EINVAL,
                   "tm_geometry_create: edge of tile %lld is not a positive number",
                   static_cast<long long>(i / 3));
    }
    tm_geom* g = new tm_geom();
    g->ctx = c;
    g->n = n;
    g->centers.assign(centers, centers + 3 * n);
    g->sizes.assign(sizes, sizes + 3 * n);
    g->hash = geometry_hash(n, centers, sizes);
    find_faces(*g);
    *out = g;
    return TM_OK;
}

tm_status tm_geometry_hash(const tm_geom* g, uint64_t* out) {
    TM_REQUIRE(g && out, TM_EINVAL, "tm_geometry_hash: null argument");
    *out = g->hash;
    return TM_OK;
}

tm_status tm_geometry_info(const tm_geom* g, int64_t* n, int64_t* nfaces) {
    TM_REQUIRE(g, TM_EINVAL, "tm_geometry_info: null geometry");
    if (n) *n = g->n;
    if (nfaces) *nfaces = static_cast<int64_t>(g->nbr_idx.size());
    return TM_OK;
}

tm_status tm_geometry_destroy(tm_geom* g) {
    TM_REQUIRE(g, TM_EINVAL, "tm_geometry_destroy: null geometry");
    delete g;
    return TM_OK;
}

tm_status tm_tensor_assemble(tm_ctx* c, const tm_geom* g, tm_prec store, tm_layout layout,
                             hipStream_t stream, tm_tensor** out) {
    TM_REQUIRE(c && g && out, TM_EINVAL, "tm_tensor_assemble: null argument");
    TM_REQUIRE(store >= TM_PREC_FP32 && store <= TM_PREC_FP64, TM_EINVAL,
               "tm_tensor_assemble: unknown precision %d", static_cast<int>(store));
    TM_REQUIRE(layout == TM_LAYOUT_SYM6 || layout == TM_LAYOUT_DENSE9 || is_psym(layout),
               TM_EINVAL, "tm_tensor_assemble: layout %d cannot be assembled", static_cast<int>(layout));
    TM_REQUIRE(layout == TM_LAYOUT_DENSE9 || store == TM_PREC_FP32 || store == TM_PREC_FP64,
               TM_EINVAL, "tm_tensor_assemble: split precisions need the DENSE9 layout");
    if (is_psym(layout)) {
        const char* nm = layout == TM_LAYOUT_PSYM4 ? "PSYM4" : "PSYM6";
        TM_REQUIRE(store == TM_PREC_FP32, TM_EINVAL, "tm_tensor_assemble: %s is stored in FP32", nm);
        for (int64_t a = 1; a < g->n; ++a)
            TM_REQUIRE(g->sizes[3 * a] == g->sizes[0] && g->sizes[3 * a + 1] == g->sizes[1] &&
                           g->sizes[3 * a + 2] == g->sizes[2],
                       TM_EINVAL, "tm_tensor_assemble: %s needs identical tiles (tile %lld differs)", nm,
                       static_cast<long long>(a));
        if (layout == TM_LAYOUT_PSYM4)
            for (int64_t a = 1; a < g->n; ++a)
                TM_REQUIRE(g->centers[3 * a + 2] == g->centers[2], TM_EINVAL,
                           "tm_tensor_assemble: PSYM4 needs one layer of tiles (tile %lld has another z)",
                           static_cast<long long>(a));
    }
    TM_TRY_HIP(hipSetDevice(c->device));
    std::unique_lock<std::mutex> lk(c->mu);
    for (auto it = c->cache.begin(); it != c->cache.end(); ++it) {
        Tensor* T = *it;
        if (T->hash == g->hash && T->prec == store && T->layout == layout && T->n == g->n &&
            T->centers == g->centers && T->sizes == g->sizes) {
            T->refs += 1;
            c->cache.splice(c->cache.begin(), c->cache, it);
            c->cache_hits += 1;
            *out = static_cast<tm_tensor*>(T);
            return TM_OK;
        }
    }
    c->cache_misses += 1;
    const int64_t n = g->n, np = padded_tiles(n);
    tm_tensor* T = new tm_tensor();
    T->ctx = c;
    T->hash = g->hash;
    T->n = n;
    T->centers = g->centers;
    T->sizes = g->sizes;
    T->prec = store;
    T->layout = layout;
    size_t esz = store == TM_PREC_FP64 ? 8 : (store == TM_PREC_FP32 ? 4 : 2);
    int64_t main_bytes = 0, lo_bytes = 0, sc_bytes = 0;
    std::vector<int32_t> pairs;
    if (is_psym(layout)) {
        // pair table: the diagonal pairs first, then I < J row by row
        T->nt = (n + kPsTile - 1) / kPsTile;
        for (int64_t I = 0; I < T->nt; ++I) {
            pairs.push_back(static_cast<int32_t>(I));
            pairs.push_back(static_cast<int32_t>(I));
        }
        for (int64_t I = 0; I < T->nt; ++I)
            for (int64_t J = I + 1; J < T->nt; ++J) {
                pairs.push_back(static_cast<int32_t>(I));
                pairs.push_back(static_cast<int32_t>(J));
            }
        T->npairs = T->nt * (T->nt + 1) / 2;
        main_bytes = T->npairs * psym_planes(layout) * kPsTile * kPsTile * 4;
        lo_bytes = 0;
    } else if (layout == TM_LAYOUT_SYM6) {
        T->ld = round_up(n, 4);
        T->plane = n * T->ld;
        T->rows = n;
        main_bytes = 6 * T->plane * static_cast<int64_t>(esz);
    } else {
        T->ld = 3 * np;
        T->rows = round_up(3 * np, 128);
        // a single layer of tiles in FP32 or split precision: the
        // component-blocked form, which leaves out the two zero blocks
        bool layer = store != TM_PREC_FP64;
        for (int64_t a = 1; a < n && layer; ++a) layer = g->centers[3 * a + 2] == g->centers[2];
        T->cblk = layer;
        main_bytes = (layer ? 5 * np * np : T->rows * T->ld) * static_cast<int64_t>(esz);
        if (store == TM_PREC_BF16X3 || store == TM_PREC_FP16X3) lo_bytes = main_bytes;
        if (store == TM_PREC_FP16X3) sc_bytes = T->rows * 4;
    }
    const int64_t pair_bytes = static_cast<int64_t>(pairs.size()) * 4;
    T->bytes = main_bytes + lo_bytes + sc_bytes + pair_bytes;
    tm_status st = admit_bytes(c, T->bytes);
    if (st != TM_OK) {
        delete T;
        return st;
    }
    auto fail = [&](tm_status code) {
        release_bytes(c, T->bytes);
        free_tensor(T);
        return code;
    };
    if (hipMalloc(&T->data, main_bytes) != hipSuccess) {
        set_error("tm_tensor_assemble: hipMalloc of %lld bytes failed", static_cast<long long>(main_bytes));
        return fail(TM_ENOMEM);
    }
    if (lo_bytes && hipMalloc(&T->lo, lo_bytes) != hipSuccess) return fail(TM_ENOMEM);
    if (sc_bytes && hipMalloc(reinterpret_cast<void**>(&T->rscale), sc_bytes) != hipSuccess)
        return fail(TM_ENOMEM);
    if (pair_bytes) {
        if (hipMalloc(reinterpret_cast<void**>(&T->pairs), pair_bytes) != hipSuccess) return fail(TM_ENOMEM);
        if (hipMemcpy(T->pairs, pairs.data(), pair_bytes, hipMemcpyHostToDevice) != hipSuccess)
            return fail(TM_EDEVICE);
    }
    double *dc = nullptr, *ds = nullptr;
    if (hipMalloc(&dc, 3 * n * sizeof(double)) != hipSuccess ||
        hipMalloc(&ds, 3 * n * sizeof(double)) != hipSuccess) {
        if (dc) (void)hipFree(dc);
        set_error("tm_tensor_assemble: geometry upload allocation failed");
        return fail(TM_ENOMEM);
    }
    hipError_t e1 = hipMemcpyAsync(dc, g->centers.data(), 3 * n * sizeof(double),
                                   hipMemcpyHostToDevice, stream);
    hipError_t e2 = hipMemcpyAsync(ds, g->sizes.data(), 3 * n * sizeof(double),
                                   hipMemcpyHostToDevice, stream);
    st = (e1 == hipSuccess && e2 == hipSuccess) ? assemble_device(T, dc, ds, stream) : TM_EDEVICE;
    hipError_t e3 = hipStreamSynchronize(stream);
    (void)hipFree(dc);
    (void)hipFree(ds);
    if (st != TM_OK) return fail(st);
    if (e3 != hipSuccess) {
        set_error("tm_tensor_assemble: %s", hipGetErrorString(e3));
        return fail(TM_EDEVICE);
    }
    T->refs = 1;
    c->cache.push_front(T);
    *out = T;
    return TM_OK;
}

tm_status tm_tensor_get(const tm_tensor* T, int64_t a, int64_t b, double out9[9]) {
    TM_REQUIRE(T && out9, TM_EINVAL, "tm_tensor_get: null argument");
    TM_REQUIRE(a >= 0 && a < T->n && b >= 0 && b < T->n, TM_EINVAL, "tm_tensor_get: index out of range");
    TM_TRY_HIP(hipSetDevice(T->ctx->device));
    if (T->layout == TM_LAYOUT_BSR6 || is_psym(T->layout)) {
        std::vector<double> row(T->n * 9);
        tm_status st = T->layout == TM_LAYOUT_BSR6 ? bsr_rows(T, a, 1, row.data()) : psym_rows(T, a, 1, row.data());
        if (st != TM_OK) return st;
        std::memcpy(out9, row.data() + b * 9, 9 * sizeof(double));
        return TM_OK;
    }
    if (T->layout == TM_LAYOUT_SYM6) {
        double v6[6];
        for (int cc = 0; cc < 6; ++cc) {
            const int64_t off = cc * T->plane + a * T->ld + b;
            if (T->prec == TM_PREC_FP64) {
                TM_TRY_HIP(hipMemcpy(&v6[cc], static_cast<const double*>(T->data) + off, 8,
                                     hipMemcpyDeviceToHost));
            } else {
                float f;
                TM_TRY_HIP(hipMemcpy(&f, static_cast<const float*>(T->data) + off, 4,
                                     hipMemcpyDeviceToHost));
                v6[cc] = f;
            }
        }
        const double m[9] = {v6[0], v6[1], v6[2], v6[1], v6[3], v6[4], v6[2], v6[4], v6[5]};
        std::memcpy(out9, m, sizeof(m));
        return TM_OK;
    }
    if (T->prec == TM_PREC_FP64) {  // row-major
        for (int i = 0; i < 3; ++i)
            TM_TRY_HIP(hipMemcpy(out9 + 3 * i, static_cast<const double*>(T->data) + (3 * a + i) * T->ld + 3 * b,
                                 24, hipMemcpyDeviceToHost));
        return TM_OK;
    }
    std::vector<double> rows(3 * T->n * 3);
    tm_status st = tm_tensor_rows(T, a, 1, rows.data());
    if (st != TM_OK) return st;
    std::memcpy(out9, rows.data() + b * 9, 9 * sizeof(double));
    return TM_OK;
}

static double half_bits_to_double(uint16_t v, bool bf16) {
    if (bf16) {
        uint32_t b = static_cast<uint32_t>(v) << 16;
        float f;
        std::memcpy(&f, &b, 4);
        return f;
    }
    __half h;
    std::memcpy(&h, &v, 2);
    return __half2float(h);
}

tm_status tm_tensor_rows(const tm_tensor* T, int64_t a0, int64_t count, double* out) {
    TM_REQUIRE(T && out, TM_EINVAL, "tm_tensor_rows: null argument");
    TM_REQUIRE(a0 >= 0 && count >= 0 && a0 + count <= T->n, TM_EINVAL, "tm_tensor_rows: rows out of range");
    if (count == 0) return TM_OK;
    TM_TRY_HIP(hipSetDevice(T->ctx->device));
    const int64_t n = T->n;
    if (T->layout == TM_LAYOUT_BSR6) return bsr_rows(T, a0, count, out);
    if (is_psym(T->layout)) return psym_rows(T, a0, count, out);
    if (T->layout == TM_LAYOUT_SYM6) {
        const size_t esz = T->prec == TM_PREC_FP64 ? 8 : 4;
        std::vector<unsigned char> buf(6 * count * T->ld * esz);
        for (int cc = 0; cc < 6; ++cc) {
            const unsigned char* src = static_cast<const unsigned char*>(T->data) +
                                       (cc * T->plane + a0 * T->ld) * esz;
            TM_TRY_HIP(hipMemcpy(buf.data() + cc * count * T->ld * esz, src, count * T->ld * esz,
                                 hipMemcpyDeviceToHost));
        }
        static const int comp[9] = {0, 1, 2, 1, 3, 4, 2, 4, 5};
        for (int64_t r = 0; r < count; ++r)
            for (int64_t b = 0; b < n; ++b)
                for (int k = 0; k < 9; ++k) {
                    const int64_t idx = comp[k] * count * T->ld + r * T->ld + b;
                    double v;
                    if (esz == 8) {
                        std::memcpy(&v, buf.data() + idx * 8, 8);
                    } else {
                        float f;
                        std::memcpy(&f, buf.data() + idx * 4, 4);
                        v = f;
                    }
                    out[(r * n + b) * 9 + k] = v;
                }
        return TM_OK;
    }
    const int64_t nrow = 3 * count;
    const int64_t r0 = 3 * a0;
    if (T->prec == TM_PREC_FP64 || T->prec == TM_PREC_FP32) {
        const size_t esz = T->prec == TM_PREC_FP64 ? 8 : 4;
        std::vector<unsigned char> buf(nrow * T->ld * esz);
        if (T->prec == TM_PREC_FP64) {
            TM_TRY_HIP(hipMemcpy(buf.data(), static_cast<const unsigned char*>(T->data) + r0 * T->ld * esz,
                                 buf.size(), hipMemcpyDeviceToHost));
        } else {
            tm_status st = dense9_rows_rowmajor(T, T->data, r0, nrow, buf.data());
            if (st != TM_OK) return st;
        }
        for (int64_t r = 0; r < count; ++r)
            for (int64_t b = 0; b < n; ++b)
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) {
                        const int64_t idx = (3 * r + i) * T->ld + 3 * b + j;
                        double v;
                        if (esz == 8) {
                            std::memcpy(&v, buf.data() + idx * 8, 8);
                        } else {
                            float f;
                            std::memcpy(&f, buf.data() + idx * 4, 4);
                            v = f;
                        }
                        out[(r * n + b) * 9 + 3 * i + j] = v;
                    }
        return TM_OK;
    }
    std::vector<uint16_t> hi(nrow * T->ld), lo(nrow * T->ld);
    std::vector<float> rs(nrow, 1.0f);
    tm_status st = dense9_rows_rowmajor(T, T->data, r0, nrow, hi.data());
    if (st == TM_OK) st = dense9_rows_rowmajor(T, T->lo, r0, nrow, lo.data());
    if (st != TM_OK) return st;
    if (T->prec == TM_PREC_FP16X3)
        TM_TRY_HIP(hipMemcpy(rs.data(), T->rscale + r0, nrow * 4, hipMemcpyDeviceToHost));
    const bool bf = T->prec == TM_PREC_BF16X3;
    for (int64_t r = 0; r < count; ++r)
        for (int64_t b = 0; b < n; ++b)
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    const int64_t idx = (3 * r + i) * T->ld + 3 * b + j;
                    out[(r * n + b) * 9 + 3 * i + j] =
                        (half_bits_to_double(hi[idx], bf) + half_bits_to_double(lo[idx], bf)) *
                        rs[3 * r + i];
                }
    return TM_OK;
}

tm_status tm_tensor_bytes(const tm_tensor* T, int64_t* bytes) {
    TM_REQUIRE(T && bytes, TM_EINVAL, "tm_tensor_bytes: null argument");
    *bytes = T->bytes;
    return TM_OK;
}

tm_status tm_tensor_release(tm_tensor* T) {
    TM_REQUIRE(T, TM_EINVAL, "tm_tensor_release: null tensor");
    std::lock_guard<std::mutex> lk(T->ctx->mu);
    TM_REQUIRE(T->refs > 0, TM_EINVAL, "tm_tensor_release: no reference held");
    T->refs -= 1;
    return TM_OK;
}

tm_status tm_problem_create(tm_ctx* c, const tm_geom* g, tm_tensor* T, const tm_material* mat,
                            tm_problem** out) {
    TM_REQUIRE(c && g && T && mat && out && mat->Ms, TM_EINVAL, "tm_problem_create: null argument");
    TM_REQUIRE(T->hash == g->hash && T->n == g->n, TM_EINVAL,
               "tm_problem_create: tensor was built from a different geometry");
    TM_REQUIRE(std::isfinite(mat->A_exch) && mat->A_exch >= 0.0, TM_EINVAL, "tm_problem_create: A_exch");
    TM_REQUIRE(std::isfinite(mat->alpha) && mat->alpha >= 0.0 && std::isfinite(mat->gamma0) &&
                   mat->gamma0 >= 0.0,
               TM_EINVAL, "tm_problem_create: alpha / gamma0");
    const int64_t n = g->n, np = padded_tiles(n);
    double msmax = 0.0;
    bool uni = true;
    for (int64_t a = 0; a < n; ++a) {
        TM_REQUIRE(std::isfinite(mat->Ms[a]) && mat->Ms[a] > 0.0, TM_EINVAL,
                   "tm_problem_create: Ms of tile %lld must be positive", static_cast<long long>(a));
        msmax = std::max(msmax, mat->Ms[a]);
        uni = uni && mat->Ms[a] == mat->Ms[0];
    }
    const bool anis = mat->Ku != nullptr;
    TM_REQUIRE(!anis || mat->easy, TM_EINVAL, "tm_problem_create: Ku given without easy axes");
    TM_TRY_HIP(hipSetDevice(c->device));

    // host-side operator pieces in float64, stored as the kernels read them
    std::vector<float> ms(np, 0.0f), w(g->nbr_idx.size()), ku, easy;
    std::vector<double> ew(n), evk(n, 0.0), xw(g->nbr_idx.size());
    for (int64_t a = 0; a < n; ++a) {
        ms[a] = static_cast<float>(mat->Ms[a]);
        const double vol = g->sizes[3 * a] * g->sizes[3 * a + 1] * g->sizes[3 * a + 2];
        ew[a] = vol * mat->Ms[a];
        for (int32_t j = g->nbr_ptr[a]; j < g->nbr_ptr[a + 1]; ++j) {
            w[j] = static_cast<float>(2.0 * mat->A_exch * g->nbr_area[j] /
                                      (kMu0 * mat->Ms[a] * vol * g->nbr_dist[j]));
            xw[j] = mat->A_exch * g->nbr_area[j] / g->nbr_dist[j];
        }
    }
    if (anis) {
        ku.resize(n);
        easy.resize(3 * n);
        for (int64_t a = 0; a < n; ++a) {
            const double* e = mat->easy + 3 * a;
            const double r = std::sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
            TM_REQUIRE(std::isfinite(mat->Ku[a]) && r > 0.0 && std::isfinite(r), TM_EINVAL,
                       "tm_problem_create: anisotropy of tile %lld", static_cast<long long>(a));
            for (int i = 0; i < 3; ++i) easy[3 * a + i] = static_cast<float>(e[i] / r);
            ku[a] = static_cast<float>(2.0 * mat->Ku[a] / (kMu0 * mat->Ms[a]));
            const double vol = g->sizes[3 * a] * g->sizes[3 * a + 1] * g->sizes[3 * a + 2];
            evk[a] = vol * mat->Ku[a];
        }
    }
    tm_problem* p = new tm_problem();
    p->ctx = c;
    p->T = T;
    p->n = n;
    p->np = np;
    p->ms_ref = msmax;
    p->uniform_ms = uni;
    if (mat->ll_form == 1) {
        p->c1 = mat->gamma0;
        p->c2 = mat->alpha;
    } else {
        p->c1 = mat->gamma0 / (1.0 + mat->alpha * mat->alpha);
        p->c2 = mat->gamma0 * mat->alpha / (1.0 + mat->alpha * mat->alpha);
    }
    const int64_t nnz = static_cast<int64_t>(g->nbr_idx.size());
    p->nnz = nnz;
    int64_t bytes = np * 4 + (n + 1) * 4 + nnz * 4 + nnz * 4 + n * 8 * 2 + nnz * 8 +
                    (anis ? n * 16 : 0);
    {
        std::lock_guard<std::mutex> lk(c->mu);
        tm_status st = admit_bytes(c, bytes);
        if (st != TM_OK) {
            delete p;
            return st;
        }
        c->live_problems += 1;
        T->refs += 1;
    }
    p->bytes = bytes;
    auto up = [](void** dst, const void* src, size_t sz) -> hipError_t {
        hipError_t e = hipMalloc(dst, sz > 0 ? sz : 4);
        if (e != hipSuccess) return e;
        return sz ? hipMemcpy(*dst, src, sz, hipMemcpyHostToDevice) : hipSuccess;
    };
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = up(reinterpret_cast<void**>(&p->Ms), ms.data(), np * 4);
    if (e == hipSuccess) e = up(reinterpret_cast<void**>(&p->nbr_ptr), g->nbr_ptr.data(), (n + 1) * 4);
    if (e == hipSuccess) e = up(reinterpret_cast<void**>(&p->nbr_idx), g->nbr_idx.data(), nnz * 4);
    if (e == hipSuccess) e = up(reinterpret_cast<void**>(&p->nbr_w), w.data(), nnz * 4);
    if (e == hipSuccess) e = up(reinterpret_cast<void**>(&p->e_w), ew.data(), n * 8);
    if (e == hipSuccess) e = up(reinterpret_cast<void**>(&p->e_vk), evk.data(), n * 8);
    if (e == hipSuccess) e = up(reinterpret_cast<void**>(&p->x_w), xw.data(), nnz * 8);
    if (anis && e == hipSuccess) e = up(reinterpret_cast<void**>(&p->ku), ku.data(), n * 4);
    if (anis && e == hipSuccess) e = up(reinterpret_cast<void**>(&p->easy), easy.data(), n * 12);
    if (e != hipSuccess) {
        set_error("tm_problem_create: %s", hipGetErrorString(e));
        tm_problem_destroy(p);
        return TM_EDEVICE;
    }
    *out = p;
    return TM_OK;
}

tm_status tm_problem_destroy(tm_problem* p) {
    TM_REQUIRE(p, TM_EINVAL, "tm_problem_destroy: null problem");
    (void)hipSetDevice(p->ctx->device);
    (void)hipDeviceSynchronize();
    int64_t wsb = p->ws ? p->ws->bytes : 0;
    p->ws.reset();
    void* ptrs[] = {p->Ms, p->nbr_ptr, p->nbr_idx, p->nbr_w, p->ku, p->easy, p->e_w, p->e_vk, p->x_w};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    {
        std::lock_guard<std::mutex> lk(p->ctx->mu);
        release_bytes(p->ctx, p->bytes + wsb);
        p->ctx->live_problems -= 1;
        p->T->refs -= 1;
    }
    delete p;
    return TM_OK;
}

}  // extern "C"

namespace tmag {

tm_status ensure_workspace(Problem* p, int64_t B) {
    const Tensor* T = p->T;
    const bool dense = T->layout == TM_LAYOUT_DENSE9 && T->prec != TM_PREC_FP64;
    if (dense)
        TM_REQUIRE(B <= kMaxGemmStates, TM_EINVAL,
                   "batched (DENSE9) path: at most %lld states per call",
                   static_cast<long long>(kMaxGemmStates));
    // the GEMM operand is read in tiles of 16 states: pad the batch
    const int64_t bcap = dense ? gemm_state_pad(T, B) : B;
    if (p->ws && p->ws->B >= bcap && (!dense || p->ws->part_splits >= gemm_splits(p))) return TM_OK;
    const int64_t np = p->np, n = p->n;
    const int64_t sb = bcap * 3 * np * 4;  // one state buffer
    const int64_t nblk = (n + 255) / 256;
    int64_t xbytes = 0, pbytes = 0, splits = 0;
    if (dense) {
        const int64_t esz = T->prec == TM_PREC_FP32 ? 4 : 2;
        // the right operand in the product's fragment order (hi + lo for the
        // split forms), once for k_prep and once per stage output ya, yb, y5
        xbytes = bcap * T->ld * esz * (T->prec == TM_PREC_FP32 ? 1 : 2);
        splits = gemm_splits(p);
        pbytes = splits * bcap * T->rows * 4;
    }
    const bool psym = is_psym(T->layout);
    if (psym) pbytes = psym_partial_floats(T, bcap) * 4;
    const int64_t dbytes = bcap * (nblk * 6 + 4) * 8;  // diagnostics partials + energies
    int64_t bytes = 12 * sb + bcap * 12 + bcap * (8 * 7 + 8 * 2 + 4 * 2 + 8 * kSnapStride + 24) + 16 * bcap * n + 576 +
                    RP_COUNT * 8 + nblk * bcap * 32 + 4 * xbytes + pbytes + dbytes;
    {
        std::lock_guard<std::mutex> lk(p->ctx->mu);
        const int64_t old = p->ws ? p->ws->bytes : 0;
        release_bytes(p->ctx, old);
        tm_status st = admit_bytes(p->ctx, bytes);
        if (st != TM_OK) {
            p->ctx->used += old;
            return st;
        }
    }
    if (p->ws) {
        (void)hipDeviceSynchronize();
        p->ws.reset();
    }
    auto w = std::make_unique<Workspace>();
    w->B = bcap;
    w->bpad = dense ? bcap : 0;
    w->bytes = bytes;
    auto alloc = [](void** d, size_t sz) -> hipError_t {
        hipError_t e = hipMalloc(d, sz);
        if (e == hipSuccess) e = hipMemset(*d, 0, sz);
        return e;
    };
    hipError_t e = hipSuccess;
    float** bufs[] = {&w->y, &w->ya, &w->yb, &w->y5, &w->hd, &w->k[0], &w->k[1], &w->k[2],
                      &w->k[3], &w->k[4], &w->k[5], &w->k[6]};
    for (float** b : bufs)
        if (e == hipSuccess) e = alloc(reinterpret_cast<void**>(b), sb);
    if (e == hipSuccess) e = alloc(reinterpret_cast<void**>(&w->Ha), bcap * 12);
    if (e == hipSuccess) e = alloc(reinterpret_cast<void**>(&w->t), bcap * 8);
    if (e == hipSuccess) e = alloc(reinterpret_cast<void**>(&w->h), bcap * 8);
    if (e == hipSuccess) e = alloc(reinterpret_cast<void**>(&w->dt), bcap * 8);
    if (e == hipSuccess) e = alloc(reinterpret_cast<void**>(&w->t1), bcap * 8);
    if (e == hipSuccess) e = alloc(reinterpret_cast<void**>(&w->h1), bcap * 8);
    if (e == hipSuccess) e = alloc(reinterpret_cast<void**>(&w->steps1), bcap * 8);
    if (e == hipSuccess) e = alloc(reinterpret_cast<void**>(&w->flags1), bcap * 4);
    w->pstride = n;  // at most one partial per target tile (one tile per block)
    if (e == hipSuccess) e = alloc(reinterpret_cast<void**>(&w->errp), bcap * n * 8);
    if (e == hipSuccess) e = alloc(reinterpret_cast<void**>(&w->dmxp), bcap * n * 8);
    if (e == hipSuccess) e = alloc(reinterpret_cast<void**>(&w->snap), bcap * kSnapStride * 8);

    if (e == hipSuccess) e = alloc(reinterpret_cast<void**>(&w->steps), bcap * 8);
    if (e == hipSuccess) e = alloc(reinterpret_cast<void**>(&w->rejected), bcap * 8);
    if (e == hipSuccess) e = alloc(reinterpret_cast<void**>(&w->flags), bcap * 4);
    if (e == hipSuccess) e = alloc(reinterpret_cast<void**>(&w->acc), bcap * 4);
    if (e == hipSuccess) e = alloc(reinterpret_cast<void**>(&w->params), RP_COUNT * 8);
    if (e == hipSuccess) e = alloc(reinterpret_cast<void**>(&w->esum), nblk * bcap * 32);
    if (e == hipSuccess) e = alloc(reinterpret_cast<void**>(&w->diag), dbytes);
    if (e == hipSuccess) e = alloc(reinterpret_cast<void**>(&w->stat), bcap * 24);
    if (e == hipSuccess) e = alloc(reinterpret_cast<void**>(&w->bar), 256);
    if (e == hipSuccess) e = alloc(reinterpret_cast<void**>(&w->bar_fail), 256);
    w->esum_blocks = nblk * bcap;
    if (dense && xbytes && e == hipSuccess) {
        const int64_t half = T->prec == TM_PREC_FP32 ? xbytes : xbytes / 2;
        e = alloc(&w->xh, half);
        if (e == hipSuccess && T->prec != TM_PREC_FP32) e = alloc(&w->xl, half);
        for (int i = 0; i < 3 && e == hipSuccess; ++i) {
            e = alloc(&w->fxh[i], half);
            if (e == hipSuccess && T->prec != TM_PREC_FP32) e = alloc(&w->fxl[i], half);
        }
    }
    if ((dense || psym) && e == hipSuccess) {
        e = alloc(reinterpret_cast<void**>(&w->part), pbytes);
        w->part_splits = splits;
    }
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&w->host_params), RP_COUNT * 8);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&w->host_flags), bcap * 4);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&w->host_steps), bcap * 8 * 2);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&w->host_stat), bcap * 24);
    if (e != hipSuccess) {
        set_error("workspace allocation (%lld bytes): %s", static_cast<long long>(bytes),
                  hipGetErrorString(e));
        std::lock_guard<std::mutex> lk(p->ctx->mu);
        release_bytes(p->ctx, bytes);
        return TM_ENOMEM;
    }
    p->ws = std::move(w);
    return TM_OK;
}

}  // namespace tmag

extern "C" {

static tm_status field_call(tm_problem* p, Epi mode, int64_t B, const float* m, const float* Ha,
                            float* out, hipStream_t s) {
    TM_REQUIRE(p && m && out && B >= 1, TM_EINVAL, "field call: bad arguments");
    TM_REQUIRE((reinterpret_cast<uintptr_t>(m) & 15) == 0 && (reinterpret_cast<uintptr_t>(out) & 15) == 0,
               TM_EINVAL, "field call: device pointers must be 16-byte aligned");
    TM_TRY_HIP(hipSetDevice(p->ctx->device));
    tm_status st = ensure_workspace(p, B);
    if (st != TM_OK) return st;
    Workspace* w = p->ws.get();
    st = launch_pack(m, B, p->n, p->np, w->ya, s);
    if (st != TM_OK) return st;
    EpiArgs e{};
    e.out = out;
    e.out_stride = 3 * p->n;
    e.Ha = Ha;
    return launch_field(p, mode, B, w->ya, e, s);
}

tm_status tm_demag(tm_problem* p, int64_t B, const float* m, float* Hd, hipStream_t s) {
    return field_call(p, Epi::HD, B, m, nullptr, Hd, s);
}

tm_status tm_heff(tm_problem* p, int64_t B, const float* m, const float* Ha, float* H, hipStream_t s) {
    return field_call(p, Epi::HEFF, B, m, Ha, H, s);
}

tm_status tm_dmdt(tm_problem* p, int64_t B, const float* m, const float* Ha, float* d, hipStream_t s) {
    return field_call(p, Epi::DMDT, B, m, Ha, d, s);
}

tm_status tm_energy(tm_problem* p, int64_t B, const float* m, const float* Ha, double* E,
                    hipStream_t s) {
    TM_REQUIRE(p && m && E && B >= 1, TM_EINVAL, "tm_energy: bad arguments");
    TM_TRY_HIP(hipSetDevice(p->ctx->device));
    tm_status st = ensure_workspace(p, B);
    if (st != TM_OK) return st;
    Workspace* w = p->ws.get();
    st = launch_pack(m, B, p->n, p->np, w->ya, s);
    if (st != TM_OK) return st;
    EpiArgs e{};
    e.out = w->hd;
    e.out_stride = 3 * p->np;
    st = launch_field(p, Epi::HD, B, w->ya, e, s);
    if (st != TM_OK) return st;
    return launch_energy(p, B, w->ya, Ha, w->hd, E, s);
}

tm_status tm_diagnostics(tm_problem* p, int64_t B, const float* m, const float* Ha, double* D,
                         hipStream_t s) {
    TM_REQUIRE(p && m && D && B >= 1, TM_EINVAL, "tm_diagnostics: bad arguments");
    TM_TRY_HIP(hipSetDevice(p->ctx->device));
    tm_status st = ensure_workspace(p, B);
    if (st != TM_OK) return st;
    Workspace* w = p->ws.get();
    st = launch_pack(m, B, p->n, p->np, w->ya, s);
    if (st != TM_OK) return st;
    EpiArgs e{};
    e.out = w->hd;
    e.out_stride = 3 * p->np;
    st = launch_field(p, Epi::HD, B, w->ya, e, s);
    if (st != TM_OK) return st;
    const int64_t nblk = (p->n + 255) / 256;
    double* E4 = w->diag + B * nblk * 6;
    st = launch_energy(p, B, w->ya, Ha, w->hd, E4, s);
    if (st != TM_OK) return st;
    EpiArgs k{};
    k.out = w->k[6];
    k.out_stride = 3 * p->np;
    k.Ha = Ha;
    st = launch_field(p, Epi::DMDT, B, w->ya, k, s);
    if (st != TM_OK) return st;
    return launch_diagnostics(p, B, w->ya, w->hd, w->k[6], E4, D, s);
}

}  // extern "C"
