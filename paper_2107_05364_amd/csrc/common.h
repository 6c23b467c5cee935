// Internal declarations of the tilemag library (not part of the C ABI).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <list>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/tilemag.h"

namespace tmag {

constexpr double kPi = 3.14159265358979323846;
constexpr double kMu0 = 4.0e-7 * kPi;  // vacuum permeability [H/m]

void set_error(const char* fmt, ...);

#define TM_TRY_HIP(call)                                                                  \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess) {                                                           \
            ::tmag::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, \
                            __LINE__);                                                    \
            return TM_EDEVICE;                                                            \
        }                                                                                 \
    } while (0)

#define TM_REQUIRE(cond, code, ...)        \
    do {                                   \
        if (!(cond)) {                     \
            ::tmag::set_error(__VA_ARGS__);  \
            return (code);                 \
        }                                  \
    } while (0)

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }
// Padded tile count of state vectors and of the dense operator: a multiple of
// 128, so that the dense operator's rows and K extent 3 np are whole numbers
// of the batched product's 128-row blocks and 64-element chunks.
inline int64_t padded_tiles(int64_t n) { return round_up(n, 128); }

// Stored order of the DENSE9 operator in FP32 / BF16X3 / FP16X3 (the MFMA
// operand of the batched product; FP64 stays row-major).  The padded
// rows x ld matrix is cut into blocks of kGemmRows x kGemmKC elements, block
// (rb, kc) at (rb * ld / kGemmKC + kc) * kGemmRows * kGemmKC, so that a block
// (one workgroup's share of one K chunk) is a contiguous span of memory.
// Inside a block the elements are in the order in which the product's lanes
// load them, every 16-byte load of a wave reading 1 KB in one piece:
//   vec = 4 (float32, 16x16x4 fragments): row 32 w + 16 rt + j, column
//     16 sub + 4 g + e at ((((w * 4 + sub) * 2 + rt) * 64 + 16 g + j) * 4 + e;
//   vec = 8 (16-bit halves, 32x32x16 fragments): row 32 w + i, column
//     16 ks + 8 q + e at (((w * 4 + ks) * 64 + 32 q + i) * 8 + e.
constexpr int kGemmRows = 128;
constexpr int kGemmKC = 64;
// Place of element (rr, kk) inside its 128 x 64 block.
__host__ __device__ inline int64_t dense9_in_block(int vec, int rr, int kk) {
    const int w = rr / 32;
    if (vec == 8) {
        const int i = rr % 32, ks = kk / 16, q = (kk % 16) / 8, e = kk % 8;
        return ((w * 4 + ks) * 64 + 32 * q + i) * 8 + e;
    }
    const int rt = (rr % 32) / 16, j = rr % 16;
    const int sub = kk / 16, g = (kk % 16) / 4, e = kk % 4;
    return (((w * 4 + sub) * 2 + rt) * 64 + 16 * g + j) * 4 + e;
}
__host__ __device__ inline int64_t dense9_index(int64_t ld, int vec, int64_t r, int64_t k) {
    const int64_t rb = r / kGemmRows, kc = k / kGemmKC;
    const int64_t base = (rb * (ld / kGemmKC) + kc) * (kGemmRows * kGemmKC);
    return base + dense9_in_block(vec, static_cast<int>(r % kGemmRows), static_cast<int>(k % kGemmKC));
}
// Component-blocked DENSE9 of a single layer of tiles (xz = yz = 0 in every
// block): rows and columns ordered by component, r' = i np + a and
// k' = j np + b for the tile-order element (3a + i, 3b + j).  The operator is
// then [[Nxx, Nxy, 0], [Nxy, Nyy, 0], [0, 0, Nzz]] in np x np blocks: the x
// and y rows (row blocks below 2np) are stored over the x and y columns
// (K in [0, 2np)), the z rows over the z columns (K in [2np, 3np)); the two
// zero parts are not stored (-1).  Blocks of 128 x 64 as dense9_index, the
// x/y rows first (2np / 64 chunks per row block), then the z rows (np / 64).
__host__ __device__ inline int64_t dense9c_index(int64_t np, int vec, int64_t r, int64_t k) {
    const int64_t a = r / 3, b = k / 3;
    const int i = static_cast<int>(r % 3), j = static_cast<int>(k % 3);
    if ((i < 2) != (j < 2)) return -1;
    const int64_t rp = i * np + a, kp = j * np + b;
    const int64_t rb = rp / kGemmRows, rb2 = 2 * np / kGemmRows;
    const int64_t kc = kp / kGemmKC, kc2 = 2 * np / kGemmKC;
    const int64_t blk = rb < rb2 ? rb * kc2 + kc : rb2 * kc2 + (rb - rb2) * (np / kGemmKC) + (kc - kc2);
    return blk * (kGemmRows * kGemmKC) +
           dense9_in_block(vec, static_cast<int>(rp % kGemmRows), static_cast<int>(kp % kGemmKC));
}

struct Tensor;

// One device; owns the tensor cache and the admission ledger.
struct Ctx {
    int device = 0;
    int64_t budget = 0;        // bytes the library may hold on the device
    int64_t used = 0;          // bytes currently held (tensors, workspaces, slots)
    std::mutex mu;
    std::list<Tensor*> cache;  // most recently used first
    int live_problems = 0;
    int live_servers = 0;
    int64_t cache_hits = 0, cache_misses = 0;
};

// Reserve / return bytes against the context budget, evicting unreferenced
// cached tensors (least recently used first) when needed.
tm_status admit_bytes(Ctx* c, int64_t bytes);
void release_bytes(Ctx* c, int64_t bytes);

struct Geom {
    Ctx* ctx = nullptr;
    int64_t n = 0;
    std::vector<double> centers, sizes;  // [n][3]
    uint64_t hash = 0;
    // ordered face-neighbour pairs in CSR form by the first tile
    std::vector<int32_t> nbr_ptr;        // [n+1]
    std::vector<int32_t> nbr_idx;
    std::vector<double> nbr_area;        // shared face area [m^2]
    std::vector<double> nbr_dist;        // centre distance along the face normal [m]
};

uint64_t geometry_hash(int64_t n, const double* centers, const double* sizes);
void find_faces(Geom& g);

struct Tensor {
    Ctx* ctx = nullptr;
    uint64_t hash = 0;
    int64_t n = 0;
    std::vector<double> centers, sizes;
    tm_prec prec = TM_PREC_FP32;
    tm_layout layout = TM_LAYOUT_SYM6;
    int64_t ld = 0;       // row stride in elements
    int64_t plane = 0;    // SYM6: stride between component planes in elements
    int64_t rows = 0;     // DENSE9: allocated rows (>= 3n)
    bool cblk = false;    // DENSE9 (FP32 / split): component-blocked single layer (dense9c_index)
    void* data = nullptr; // fp32 / fp64 entries, or the hi part
    void* lo = nullptr;   // lo part of split precisions
    float* rscale = nullptr; // FP16X3: per-row 1/scale (power of two)
    // BSR6 (thresholded): data = float [6][nnzb] components, row_ptr [n+1],
    // col [nnzb] source tiles in ascending order per row
    int64_t* row_ptr = nullptr;
    int32_t* col = nullptr;
    int64_t nnzb = 0;
    // PSYM6 (pair-symmetric): data = float [npairs][6][kPsTile][kPsTile] tiles of the
    // upper triangle, pairs = int32 [npairs][2] (I, J), I <= J, nt tiles a side;
    // PSYM4 the same with the planes (xx, xy, yy, zz) of a single layer of tiles
    int32_t* pairs = nullptr;
    int64_t npairs = 0, nt = 0;
    int bsr_planes = 6;      // BSR6: component planes stored (4 for a single layer: xz = yz = 0)
    double frac = -1.0;      // BSR6: removed fraction requested
    double cut = -1.0;       // BSR6: magnitude cut (-1: nothing removed)
    int64_t bytes = 0;
    int refs = 0;
};

// Pair-symmetric layouts and their stored planes.
inline bool is_psym(int layout) { return layout == TM_LAYOUT_PSYM6 || layout == TM_LAYOUT_PSYM4; }
inline int psym_planes(int layout) { return layout == TM_LAYOUT_PSYM4 ? 4 : 6; }

// Frees a tensor's device memory and the tensor (the ledger is the caller's).
void free_tensor(Tensor* T);

// Device-side description of the pieces of a problem the kernels read.
struct DevProblem {
    int32_t n;          // tiles
    int32_t np;         // padded tile count (multiple of 4); state stride = 3*np floats
    const float* Ms;    // [np] saturation magnetisation, 0 in the padding
    const int32_t* nbr_ptr;
    const int32_t* nbr_idx;
    const float* nbr_w; // 2A S_ab / (mu0 Ms_a V_a d_ab)  [A/m per unit of m]
    const float* ku;    // [n] 2K/(mu0 Ms) or nullptr
    const float* easy;  // [n][3] unit axes or nullptr
    float c1, c2;       // LL coefficients
};

struct Workspace;

struct Problem {
    Ctx* ctx = nullptr;
    Tensor* T = nullptr;
    int64_t n = 0, np = 0;
    double c1 = 0, c2 = 0;
    double ms_ref = 0;          // max Ms (scale of the GEMM right operand)
    bool uniform_ms = true;
    // device arrays
    float* Ms = nullptr;
    int32_t* nbr_ptr = nullptr;
    int32_t* nbr_idx = nullptr;
    float* nbr_w = nullptr;
    float* ku = nullptr;
    float* easy = nullptr;
    double* e_w = nullptr;      // [n] V_a Ms_a (float64, energy weights)
    double* e_vk = nullptr;     // [n] V_a K_a
    double* x_w = nullptr;      // per face A S/d (exchange energy), same CSR
    int64_t nnz = 0;
    int shape = -1;             // field-kernel launch shape (-1: default for n)
    int gemm_splits = 0;        // batched product: K splits (0: default for the operator)
    int psym_nt = -1;           // pair-symmetric tile pass: nontemporal operator loads (1) or
                                // cached (0); -1: by operator size
    int64_t bytes = 0;          // device bytes owned by the problem
    std::unique_ptr<Workspace> ws;
    DevProblem dev() const;
};

// Integrator / field workspace sized for a batch of B states.
struct Workspace {
    int64_t B = 0;
    int64_t bytes = 0;
    float* y = nullptr;       // [B][np][3] current state
    float* ya = nullptr;      // stage input buffers
    float* yb = nullptr;
    float* y5 = nullptr;      // fifth-order solution (DP45) / scratch
    float* k[7] = {};         // stage derivatives
    float* Ha = nullptr;      // [B][3]
    float* hd = nullptr;      // [B][np][3] demag / field scratch
    // GEMM operands and partial sums (batched path)
    void* xh = nullptr;       // right operand hi  [B][ld3]
    void* xl = nullptr;       // right operand lo
    float* part = nullptr;    // split-K partials [S][bpad][rows]
    int64_t part_splits = 0;
    int64_t bpad = 0;         // states in the GEMM operand buffers (multiple of 16)
    // the right operand of ya, yb and y5 in the same order, written by the
    // stage whose output they are (zero in the padding: allocated zeroed,
    // never written there).  frag_src: the buffer whose copy the last
    // batched launch wrote (else null); frag_chain: set by a caller whose
    // next launch reads the previous stage's output unchanged (the stages
    // of one attempt), so that that launch may use the copy
    void* fxh[3] = {};
    void* fxl[3] = {};
    const float* frag_src = nullptr;
    bool frag_chain = false;
    // per-state control
    double* t = nullptr;
    double* h = nullptr;      // step used by the current attempt (0: frozen)
    double* dt = nullptr;     // proposal
    // a second set of RK4 control values (t, h, steps, flags): an attempt
    // whose last stage advances the control writes it, the next one reads it
    double* t1 = nullptr;
    double* h1 = nullptr;
    int64_t* steps1 = nullptr;
    int32_t* flags1 = nullptr;
    double* errp = nullptr;   // [B][pstride] per-block maxima of the scaled error
    double* dmxp = nullptr;   // [B][pstride] per-block maxima of |dm/dt|
    int64_t pstride = 0;
    double* snap = nullptr;   // [B][kSnapStride] control values as the last stage saw them

    int64_t* steps = nullptr;
    int64_t* rejected = nullptr;
    int32_t* flags = nullptr;
    int32_t* acc = nullptr;
    double* params = nullptr; // RunParams on device
    double* esum = nullptr;   // energy partial sums
    double* diag = nullptr;   // diagnostics: [B][nblk][6] partials, then [B][4] energies
    int64_t* stat = nullptr;  // end of a run: [3][B] accepted steps, rejected attempts, flags
    unsigned* bar = nullptr;  // persistent RK4: grid-barrier counter
    int32_t* bar_fail = nullptr;  // persistent RK4: a barrier wait gave up
    int64_t esum_blocks = 0;
    // pinned host mirrors (run parameters, polling)
    double* host_params = nullptr;
    int32_t* host_flags = nullptr;
    int64_t* host_steps = nullptr;
    int64_t* host_stat = nullptr;  // pinned mirror of stat
    // captured step graphs: one attempt, 2, 4 and 8 attempts, and kGraphSteps
    // attempts (a run of c attempts replays at most one of each below
    // kGraphSteps: each replay costs a few microseconds of its own)
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t graph1 = nullptr;
    hipGraphExec_t graphP[3] = {nullptr, nullptr, nullptr};
    hipGraphExec_t graphK = nullptr;
    int graph_integ = -1;       // scheme, batch and renormalisation the graphs were captured for
    int64_t graph_B = -1;
    int graph_renorm = -1;
    void drop_graphs();  // destroys the step graphs (they hold launch shapes and kernels)
    ~Workspace();
};

tm_status ensure_workspace(Problem* p, int64_t B);
// Device address of the fixed scratch buffer of tm_demag_noalloc on `device`,
// looked up once per device (noalloc.hip); called by tm_init.
tm_status noalloc_setup(int device);
constexpr int kGraphSteps = 16;  // a power of two: the remainder of a run is replayed from the 1, 2, 4, 8 graphs
static_assert(kGraphSteps == 16, "the step graphs cover remainders below 16 attempts");
// A state's control snapshot: h, t and dt, then the step counts and the
// flags as 64-bit integer bit patterns.
enum SnapSlot : int { SN_H = 0, SN_T = 1, SN_DT = 2, SN_STEPS = 3, SN_REJ = 4, SN_FLAGS = 5 };
constexpr int kSnapStride = 8;

// Durations of the operator-pass launches inside an integration
// (tm_profile_run).  While a timer is installed on the calling thread, the
// launchers of the operator kernels (k_field, k_psym_tiles, k_field_bsr, the
// batched products) take the next pair of events and launch through
// hipExtLaunchKernelGGL, which stamps the kernel's own start and end on them;
// once the pairs run out they launch plainly.
struct OpTimer {
    std::vector<hipEvent_t> ev;  // two per launch
    int64_t used = 0;            // launches stamped
};
OpTimer*& op_timer();  // the calling thread's timer (nullptr: none)

template <typename... Formals, typename... Actuals>
inline void launch_op(void (*kernel)(Formals...), dim3 grid, dim3 block, hipStream_t s, Actuals... args) {
    OpTimer* t = op_timer();
    if (t && 2 * t->used + 1 < static_cast<int64_t>(t->ev.size())) {
        hipExtLaunchKernelGGL(kernel, grid, block, 0, s, t->ev[2 * t->used], t->ev[2 * t->used + 1], 0,
                              static_cast<Formals>(args)...);
        ++t->used;
    } else {
        kernel<<<grid, block, 0, s>>>(args...);
    }
}

// Kernel launchers (fieldstep.hip).
enum class Epi : int { HD = 0, HEFF = 1, DMDT = 2, STAGE = 3, RK4_FINAL = 4, DP_LAST = 5 };

struct EpiArgs {
    float* out;            // HD/HEFF/DMDT: output; STAGE/DP_LAST: k of this stage
    int64_t out_stride;    // floats between states of `out`
    const float* Ha;       // [B][3] or nullptr
    const float* y;        // base state (STAGE, RK4_FINAL, DP_LAST)
    float* y_mut;          // RK4_FINAL: state updated in place
    const float* kprev[6]; // previous stage derivatives
    float coef[7];         // STAGE: next-input weights of kprev[0..nprev-1] and of this k
    int32_t nprev;
    float* ynext;          // STAGE: next stage input
    const double* h;       // [B] step of this attempt
    const double* params;  // RunParams (atol, rtol, ...)
    double* errp;          // DP_LAST: per-block partial maxima, [B][pstride]
    double* dmxp;
    int64_t pstride;
    int32_t renorm;
    // DP_LAST: the control values of each state (t, dt, step counts, flags;
    // h above) and where the first block of the state copies them for the
    // commit pass, [B][kSnapStride]
    const double* t;
    const double* dt;
    const int64_t* steps;
    const int64_t* rejected;
    const int32_t* flags;
    double* snap;
    // RK4_FINAL with rk_t_out set: the first workgroup of each state also
    // advances the RK4 step control from the values the stages read (t, h,
    // steps, flags above) into this second set, which the next attempt reads
    double* rk_t_out;
    double* rk_h_out;
    int64_t* rk_steps_out;
    int32_t* rk_flags_out;
};

// H (or a stage) for B states whose inputs X are padded internal buffers.
tm_status launch_field(const Problem* p, Epi mode, int64_t B, const float* X, const EpiArgs& e,
                       hipStream_t s);
// Batched (MFMA GEMM) path for DENSE9 operators (gemm.hip).
// Host copy of rows [r0, r0 + nrow) of a blocked DENSE9 array (src = the
// hi, lo or float32 data of T), row-major, nrow x ld elements.
tm_status dense9_rows_rowmajor(const Tensor* T, const void* src, int64_t r0, int64_t nrow, void* host);
int gemm_state_tiles(int64_t B);
// States of a batched-product call padded to the product's state tiles
// (float32: 16 x {1, 2, 4, 8}; the split forms: 32 x {1, 2, 4}).
int64_t gemm_state_pad(const Tensor* T, int64_t B);
int64_t gemm_splits(const Problem* p);
// Batched product: choices from kGemmAligned on are the aligned work plan
// with choice - kGemmAligned K super-ranges (component-blocked operators
// whose parts fit it); the plan's super-range count, else 0.
constexpr int kGemmAligned = 100;
int gemm_aligned_nq(const Problem* p, int choice);
tm_status launch_field_batched(const Problem* p, Epi mode, int64_t B, const float* X,
                               const EpiArgs& e, hipStream_t s);
constexpr int64_t kMaxGemmStates = 128;
// Thresholded (BSR6) operators (threshold.hip): field kernel and host read-back.
tm_status launch_field_bsr(const Problem* p, Epi mode, int64_t B, const float* X, const EpiArgs& e,
                           hipStream_t s);
tm_status bsr_rows(const Tensor* T, int64_t a0, int64_t count, double* out);
// Pair-symmetric (PSYM6) operators (psym.hip): tiles of kPsTile x kPsTile
// blocks; assembly, field kernels (tile pass + fixed-order reduction with the
// epilogue), partial-buffer size and host read-back.
constexpr int kPsTile = 32;
tm_status assemble_psym(Tensor* T, const double* d_centers, const double* d_sizes, hipStream_t s);
tm_status launch_field_psym(const Problem* p, Epi mode, int64_t B, const float* X, const EpiArgs& e,
                            hipStream_t s);
// The same with the slot sums in a caller-provided buffer of
// psym_partial_floats(T, B) floats instead of the problem's workspace.
tm_status launch_field_psym_slots(const Problem* p, Epi mode, int64_t B, const float* X, const EpiArgs& e,
                                  float* part, hipStream_t s);
int64_t psym_partial_floats(const Tensor* T, int64_t B);
tm_status launch_psym_tiles(const Problem* p, int64_t B, const float* X, const double* h, const float* Ha,
                            hipStream_t s);
tm_status psym_rows(const Tensor* T, int64_t a0, int64_t count, double* out);

// Launch shapes of the fused field kernel: (index, workgroup threads,
// target tiles per workgroup, nontemporal operator loads, waves-per-SIMD cap).
#define TM_FIELD_SHAPES(X)        \
    X(0, 64, 2, 0, 8)             \
    X(1, 128, 2, 0, 8)            \
    X(2, 128, 4, 0, 8)            \
    X(3, 256, 2, 0, 8)            \
    X(4, 256, 4, 0, 8)            \
    X(5, 256, 8, 0, 8)            \
    X(6, 512, 4, 0, 8)            \
    X(7, 512, 8, 0, 8)            \
    X(8, 256, 2, 1, 8)            \
    X(9, 256, 4, 1, 8)            \
    X(10, 128, 1, 0, 8)           \
    X(11, 256, 1, 0, 8)           \
    X(12, 256, 4, 0, 2)           \
    X(13, 256, 8, 0, 2)           \
    X(14, 128, 4, 0, 2)           \
    X(15, 512, 8, 0, 2)           \
    X(16, 256, 1, 1, 8)           \
    X(17, 128, 1, 1, 8)           \
    X(18, 256, 4, 1, 2)           \
    X(19, 256, 8, 1, 2)
constexpr int kNumShapes = 20;
int default_shape(int64_t n);
tm_status launch_pack(const float* src, int64_t B, int64_t n, int64_t np, float* dst, hipStream_t s);
tm_status launch_control(Workspace* w, int64_t B, int integ, hipStream_t s);
tm_status launch_commit(const Problem* p, Workspace* w, int64_t B, hipStream_t s);
// blocks per state of the last-stage launch = partial maxima to reduce
int64_t last_stage_blocks(const Problem* p);
tm_status launch_energy(const Problem* p, int64_t B, const float* X, const float* Ha,
                        const float* Hd, double* E, hipStream_t s);
// Mean moment, max |dm/dt| and non-finite flag of each state; D [B][9] gets
// the energies E4 [B][4] in 0..3 (fieldstep.hip).
tm_status launch_diagnostics(const Problem* p, int64_t B, const float* X, const float* Hd,
                             const float* dmdt, const double* E4, double* D, hipStream_t s);

// Autotuner cache (tunecache.cpp): a process-wide table of tm_problem_tune
// results keyed by device, layout, precision, tile count and batch.
struct TuneResult {
    int choice = -1;
    double ms = 0.0;
};
bool tune_lookup(const Problem* p, int64_t B, TuneResult* out);
void tune_store(const Problem* p, int64_t B, const TuneResult& r);

// Persistent RK4 (persist.hip): one cooperative launch integrates one state
// whose FP32 SYM6 operator rows fit in the LDS of the workgroups.
constexpr int64_t kPersistMaxTiles = 1024;  // padded tiles
bool persistent_eligible(const Problem* p, int integ, int64_t B);
tm_status launch_persistent_rk4(const Problem* p, Workspace* w, const tm_run_cfg* cfg, hipStream_t s);

// Integrator pieces shared with the server (integrate.hip).
tm_status enqueue_attempts(const Problem* p, Workspace* w, int integ, int64_t B, int renorm,
                           int count, hipStream_t s);
tm_status capture(const Problem* p, Workspace* w, int integ, int64_t B, int renorm, int count,
                  hipGraphExec_t* out);
tm_status start_slot(const Problem* p, Workspace* w, int64_t i, double dt0, hipStream_t s);
tm_status free_slot(Workspace* w, int64_t i, hipStream_t s);

// Run-parameter slots stored in Workspace::params (doubles).
enum RunParam { RP_ATOL = 0, RP_RTOL, RP_TEND, RP_DTMIN, RP_DMDT_STOP, RP_MAX_STEPS, RP_RENORM,
                RP_COUNT };

// Per-state flag bits.
constexpr int32_t FLAG_DONE = 1, FLAG_NONFINITE = 2, FLAG_STEP = 4, FLAG_CAPPED = 8;

}  // namespace tmag

// The opaque handles of the C ABI are the library's own objects.
struct tm_ctx : tmag::Ctx {};
struct tm_geom : tmag::Geom {};
struct tm_tensor : tmag::Tensor {};
struct tm_problem : tmag::Problem {};

