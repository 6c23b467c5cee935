/*
 * tilemag.h -- C ABI of the tile micromagnetics library for AMD MI355X (gfx950).
 *
 * The library evaluates the hot path of the analytical-demagnetisation-tensor
 * method of Bjork, Poulsen, Nielsen & Insinga, "MagTense: a micromagnetic
 * framework using the analytical demagnetization tensor", J. Magn. Magn.
 * Mater. 535, 168057 (2021):
 *   - the domain is split into N uniformly magnetised cuboid tiles and the
 *     state is the 3N vector m (Sec. 3);
 *   - the demag field at each tile centre is the superposition of the
 *     analytical fields of all tiles, H_d = -N (Ms m), with a dense 3N x 3N
 *     operator computed once (Sec. 3, Sec. 3.1, Sec. 3.2);
 *   - the effective field adds exchange (finite differences, Neumann
 *     boundary), uniaxial anisotropy and the applied field (Sec. 2.1, 2.3);
 *   - the Landau-Lifshitz equation is integrated with an explicit Runge-Kutta
 *     (4,5) pair (Sec. 2.1 eq. LL, Sec. 3.1).
 *
 * Conventions (apply to every entry point):
 *   - Every call returns tm_status: TM_OK (0) or a negative code.  The text of
 *     the last error on the calling thread is returned by tm_last_error().
 *   - SI units: lengths in m, Ms and fields in A/m, A in J/m, K in J/m^3,
 *     time in s, energies in J.
 *   - Host arrays are owned by the caller and copied during the call.
 *   - Device pointers are owned by the caller, borrowed for the call and used
 *     in stream order on the given stream; calls return after enqueueing
 *     unless stated otherwise.  Device pointers must be 16-byte aligned.
 *   - State arrays are float32 [B][N][3] (state-major, tile, component),
 *     applied fields float32 [B][3].
 *   - Opaque handles are created and destroyed only by the library.  A
 *     handle may be used from one thread at a time.
 *   - HIP runtime errors are reported as TM_EDEVICE with the HIP message.
 */
#ifndef TILEMAG_H
#define TILEMAG_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t tm_status;
#define TM_OK 0
#define TM_EINVAL (-1)      /* invalid argument (shape, null pointer, non-finite input) */
#define TM_ENOMEM (-2)      /* device allocation failed or admission budget exceeded */
#define TM_EDEVICE (-3)     /* HIP runtime error */
#define TM_ENONFINITE (-4)  /* a state produced a non-finite value */
#define TM_ESTEP (-5)       /* step size underflow or attempt limit reached */
#define TM_EBUSY (-6)       /* resource still in use */
#define TM_ENOTFOUND (-7)   /* unknown ticket or handle */

/* Storage precision of the demag operator. */
typedef enum {
    TM_PREC_FP32 = 0,    /* float32 entries, float32 products */
    TM_PREC_BF16X3 = 1,  /* bf16 hi + lo entries; MFMA hi*hi + hi*lo + lo*hi, fp32 accumulate */
    TM_PREC_FP16X3 = 2,  /* fp16 hi + lo entries with a power-of-two scale per row */
    TM_PREC_FP64 = 3     /* float64 entries (verification and debugging only) */
} tm_prec;

/* Layout of the stored operator. */
typedef enum {
    TM_LAYOUT_SYM6 = 0,   /* 6 planes [6][N][ldN] of (xx,xy,xz,yy,yz,zz), each 3x3 block symmetric */
    TM_LAYOUT_DENSE9 = 1, /* dense [3N][ld3N] operator, the MFMA GEMM operand: FP64 row-major;
                             FP32 and the split forms in blocks of 128 rows x 64 columns
                             ordered as the product loads them (read back row-major); for a
                             single layer of tiles (one z for every centre) FP32 and the split
                             forms order rows and columns by component and leave out the two
                             blocks that vanish there (xz and yz): 5/9 of the bytes and
                             products */
    TM_LAYOUT_BSR6 = 2,   /* thresholded operator: block-sparse rows of 6-component blocks
                             (made by tm_tensor_threshold only) */
    TM_LAYOUT_PSYM6 = 3,  /* pair-symmetric operator of a mesh of identical tiles: only the
                             upper triangle of 32x32-block tiles, [pairs][6][32][32], since
                             N^{ab} = N^{ba} there (about half the SYM6 bytes) */
    TM_LAYOUT_PSYM4 = 4   /* PSYM6 for a single layer of identical tiles (one z for every
                             centre): xz and yz vanish there, so the tiles hold the four
                             planes (xx,xy,yy,zz), [pairs][4][32][32] (two thirds of PSYM6) */
} tm_layout;

typedef enum { TM_RK4 = 0, TM_DP45 = 1 } tm_integrator;

typedef struct tm_ctx tm_ctx;
typedef struct tm_geom tm_geom;
typedef struct tm_tensor tm_tensor;
typedef struct tm_problem tm_problem;
typedef struct tm_server tm_server;

/* Text of the last error raised on the calling thread ("" if none).  The
 * pointer stays valid until the next call on that thread. */
const char* tm_last_error(void);

/* Library version as major*10000 + minor*100 + patch. */
int32_t tm_version(void);

/* Probe rates of device `device`, measured with the library's own kernels
 * (context for the roofline fractions, which use published peaks; not
 * ceilings: a well-shaped kernel can stream faster than the read probe):
 * a streaming read of a zero-filled read_bytes buffer (1 MiB .. 16 GiB,
 * rounded down to whole 64 KiB chunks; allocated and freed by the call) in
 * GB/s, the fastest of: one workgroup per chunk as the pair-symmetric tile
 * pass reads its tiles, and one long contiguous stream per workgroup (2, 4 or
 * 8 workgroups per CU) as the stage kernel reads its rows, each with cached
 * and with nontemporal loads; and register-only loops of the
 * 32x32x16 bf16 and 16x16x4 float32 MFMA instructions the batched product
 * issues, in TFLOP/s.  Output pointers may be NULL (that measurement is
 * skipped).  Blocking; uses the device's null stream.  TM_EINVAL for a size
 * out of range, TM_EDEVICE on a HIP error. */
tm_status tm_measure_peaks(int32_t device, int64_t read_bytes, double* read_gbs, double* mfma_bf16_tflops,
                           double* mfma_fp32_tflops);

/* Opens device `device` (HIP ordinal) and creates a context that owns the
 * tensor cache and the admission budget (default: free device memory at
 * creation minus 4 GiB).  TM_EDEVICE if the device cannot be opened. */
tm_status tm_init(int32_t device, tm_ctx** out);

/* Destroys the context and every tensor it owns.  TM_EBUSY if problems or
 * servers created from it still exist. */
tm_status tm_finalize(tm_ctx* ctx);

/* Sets the admission budget in bytes for library-owned device memory
 * (tensors, integrator workspaces, server slots). */
tm_status tm_set_memory_budget(tm_ctx* ctx, int64_t bytes);

/* Geometry of N axis-aligned cuboid tiles (paper Sec. 3).  Host-side only:
 * ctx may be NULL (the geometry touches no device).
 *   centers: host [n][3] tile centres [m]
 *   sizes  : host [n][3] full edge lengths [m], all > 0
 * The tiles must not overlap.  Also finds the face-sharing neighbour pairs
 * used by the exchange operator.  TM_EINVAL on n < 1, a null pointer, a
 * non-finite value or a non-positive edge. */
tm_status tm_geometry_create(tm_ctx* ctx, int64_t n, const double* centers, const double* sizes,
                             tm_geom** out);

/* 64-bit hash of the canonical geometry bytes (n, centres, edges); equal
 * geometries hash equal.  The tensor cache keys on it and confirms hits by
 * comparing the bytes. */
tm_status tm_geometry_hash(const tm_geom* g, uint64_t* out);

/* Number of tiles and number of ordered face-neighbour pairs. */
tm_status tm_geometry_info(const tm_geom* g, int64_t* n, int64_t* nfaces);

tm_status tm_geometry_destroy(tm_geom* g);

/* Assembles (or finds in the context's cache) the dense demag operator of g:
 * block (a, b) is the analytical tensor of tile b at the centre of tile a
 * (paper Sec. 3), evaluated in float64 on the device and stored in
 * `store` precision and `layout`.  FP32 and FP64 support SYM6 and DENSE9;
 * BF16X3 and FP16X3 require DENSE9.  PSYM6 (FP32 only) stores each
 * symmetric pair of blocks once, which the paper's symmetry remark
 * (Sec. 3.2) allows when all tiles are identical: it requires every tile to
 * have the same edges (TM_EINVAL otherwise).  PSYM4 further requires every
 * centre to have the same z: the tensor of a tile at a point of its own
 * mid-plane is even in z, so its xz and yz components are zero for every
 * pair and are not stored (tm_tensor_get returns them as 0).  The returned handle holds a reference;
 * release it with tm_tensor_release.  The call blocks until the operator is
 * ready.  TM_ENOMEM if it does not fit the admission budget after evicting
 * unreferenced cached tensors. */
tm_status tm_tensor_assemble(tm_ctx* ctx, const tm_geom* g, tm_prec store, tm_layout layout,
                             hipStream_t stream, tm_tensor** out);

/* Thresholded operator (paper Sec. 4.3.1: the smallest fraction of the
 * nonzero tensor entries is set to zero and the rest is kept as a sparse
 * matrix).  `src` must be an FP32 SYM6 operator; `frac` in [0, 1].
 * Ranking: the float32 magnitudes of all 9 entries of every 3x3 block (self
 * blocks included) that are nonzero -- above 1e-14, the float64 assembly's
 * absolute rounding level -- K of them; the cut is the
 * ceil(frac K)-th smallest; every entry whose magnitude is at most the cut is
 * set to zero (ties at the cut included), except in self blocks (a == b),
 * which are kept whole.  frac = 0 removes nothing.
 * The result is a new operator of layout TM_LAYOUT_BSR6, precision FP32: for
 * each target tile, in ascending source order, the source tiles whose block
 * keeps at least one entry, with its 6 components (removed ones are 0); on a
 * single layer of tiles (one z for every centre), where xz = yz = 0 in every
 * block, only the planes xx, xy, yy, zz are stored (20 instead of 28 bytes
 * per block; read-back returns xz = yz = 0).  It
 * is usable wherever an FP32 SYM6 operator is (tm_problem_create, one state
 * or many; not the DENSE9 batched product), is cached under (geometry, frac)
 * and is released with tm_tensor_release.  Blocking.
 * Errors: TM_EINVAL (src not FP32 SYM6, frac outside [0, 1]), TM_ENOMEM. */
tm_status tm_tensor_threshold(tm_ctx* ctx, const tm_tensor* src, double frac, hipStream_t stream,
                              tm_tensor** out);

/* Size of a BSR6 operator: stored blocks and the cut (the float32 magnitude
 * at or below which entries were removed; -1 when none was). */
tm_status tm_tensor_sparse_info(const tm_tensor* t, int64_t* nnzb, double* cut);

/* Copies a BSR6 operator to host memory: row_ptr [n+1] (int64), col [nnzb]
 * source tiles (int32), vals [6][nnzb] components (xx,xy,xz,yy,yz,zz), each
 * caller-allocated.  Blocking.  TM_EINVAL for other layouts. */
tm_status tm_tensor_sparse_get(const tm_tensor* t, int64_t* row_ptr, int32_t* col, float* vals);

/* Reads back block (a, b) as stored (converted to double), row-major 3x3.
 * Blocking.  For split precisions returns (hi + lo) / scale; for BSR6 the
 * block if stored, else zeros. */
tm_status tm_tensor_get(const tm_tensor* t, int64_t a, int64_t b, double out9[9]);

/* Reads back the blocks of target tiles [a0, a0 + count) against every
 * source tile, as stored (converted to double; split precisions as
 * (hi + lo) / scale; BSR6 blocks not stored as zeros), into host
 * out[count][n][9] (row-major 3x3 blocks).  Blocking. */
tm_status tm_tensor_rows(const tm_tensor* t, int64_t a0, int64_t count, double* out);

/* Device bytes held by the stored operator. */
tm_status tm_tensor_bytes(const tm_tensor* t, int64_t* bytes);

/* Drops the caller's reference; the tensor stays cached until evicted. */
tm_status tm_tensor_release(tm_tensor* t);

/* Material data (paper Sec. 2.1-2.3).
 *   Ms     : host [n] saturation magnetisation [A/m], > 0 (required)
 *   A_exch : exchange constant [J/m], >= 0
 *   Ku     : host [n] uniaxial anisotropy constant [J/m^3] or NULL (none)
 *   easy   : host [n][3] easy axes (normalised by the library) or NULL
 *   alpha, gamma0, ll_form: Landau-Lifshitz coefficients of
 *            dm/dt = -c1 m x H - c2 m x (m x H):
 *            ll_form 0: alpha is the Gilbert damping,
 *                       c1 = gamma0/(1+alpha^2), c2 = gamma0 alpha/(1+alpha^2);
 *            ll_form 1: c1 = gamma0, c2 = alpha (the paper's LL parameters). */
typedef struct {
    const double* Ms;
    double A_exch;
    const double* Ku;
    const double* easy;
    double alpha;
    double gamma0;
    int32_t ll_form;
} tm_material;

/* Binds geometry, operator and material into a problem.  The problem keeps a
 * reference to the tensor.  `g` must be the geometry the tensor was built
 * from (checked by hash). */
tm_status tm_problem_create(tm_ctx* ctx, const tm_geom* g, tm_tensor* t, const tm_material* mat,
                            tm_problem** out);
tm_status tm_problem_destroy(tm_problem* p);

/* H_d = -N (Ms m) for B states (paper Sec. 2.3 demag term, Sec. 3.1).
 *   m : device [B][n][3] float32,  Hd : device [B][n][3] float32 [A/m]. */
tm_status tm_demag(tm_problem* p, int64_t B, const float* m, float* Hd, hipStream_t stream);

/* H_eff = H_d + H_ex + H_anis + H_a (paper Sec. 2.3, affine form of Sec. 3.1).
 *   Ha : device [B][3] applied field [A/m] (NULL: zero). */
tm_status tm_heff(tm_problem* p, int64_t B, const float* m, const float* Ha, float* H,
                  hipStream_t stream);

/* dm/dt = -c1 m x H_eff - c2 m x (m x H_eff) (paper Sec. 2.1) [1/s]. */
tm_status tm_dmdt(tm_problem* p, int64_t B, const float* m, const float* Ha, float* dmdt,
                  hipStream_t stream);

/* Free energy terms per state [J] (paper Sec. 2.2-2.3), accumulated in
 * float64: E[b][0] demag, [1] exchange, [2] anisotropy, [3] Zeeman.
 *   E : device [B][4] float64. */
tm_status tm_energy(tm_problem* p, int64_t B, const float* m, const float* Ha, double* E,
                    hipStream_t stream);

/* Diagnostics per state, accumulated in float64 in a fixed order:
 *   D[b][0..3] the energy terms as tm_energy [J];
 *   D[b][4..6] the mean magnetisation <m> = sum_a V_a Ms_a m_a / sum_a V_a Ms_a
 *              (the normalised total moment; the volume average when Ms is
 *              uniform);
 *   D[b][7]    max_a |dm/dt|_a [1/s] (paper Sec. 2.1: zero at equilibrium);
 *   D[b][8]    1 if any component of m, H_d or dm/dt of the state is not
 *              finite, else 0.
 *   D : device [B][9] float64.  Stream-ordered. */
tm_status tm_diagnostics(tm_problem* p, int64_t B, const float* m, const float* Ha, double* D,
                         hipStream_t stream);

/* Integration controls. */
typedef struct {
    int64_t max_steps;     /* accepted steps per state (RK4: steps) */
    int64_t max_attempts;  /* > 0: replay exactly this many attempted steps; 0: until done */
    double t_end;          /* > 0: stop each state at t = t_end */
    double atol, rtol;     /* DP45 error tolerances (max norm) */
    double dt_min;         /* DP45: a state whose step falls below this fails with TM_ESTEP */
    double dmdt_stop;      /* > 0: a state is done once max_a |dm/dt|_a < dmdt_stop [1/s] */
    int32_t renorm;        /* 1: |m_a| := 1 after each accepted step */
    int32_t use_graph;     /* 1: capture one attempted step in a hipGraph and replay it */
    int32_t poll_every;    /* attempts between host checks of the done flags (0: 64) */
    int32_t persistent;    /* 1: RK4 of one state with an FP32 SYM6 operator of at most 1024
                              tiles as one cooperative launch for the whole run (each
                              workgroup keeps its operator rows in LDS, a grid barrier
                              ends each stage); TM_EINVAL for any other case */
} tm_run_cfg;

typedef struct {
    int64_t attempts;      /* attempted steps replayed (all states together) */
    int64_t accepted_min;  /* fewest accepted steps over the states */
    int64_t accepted_max;
    int64_t rejected;      /* rejected attempts summed over states */
    int32_t states_done;   /* states that reached max_steps, t_end or dmdt_stop */
    int32_t states_failed; /* states stopped by a non-finite value or step underflow */
    double elapsed_ms;     /* host wall time of the call */
} tm_run_stats;

/* Integrates B independent states that share the problem's operator
 * (paper Sec. 3.1: explicit Runge-Kutta (4,5); RK4 with fixed dt).
 *   m  : device [B][n][3] float32, initial state in, final state out
 *   Ha : device [B][3] applied field per state (NULL: zero)
 *   t  : device [B] float64 time, in/out
 *   dt : device [B] float64 step size (RK4: fixed step; DP45: initial and
 *        final proposal), in/out
 *   steps_out : device [B] int64 accepted steps per state, or NULL
 * Blocks until finished.  Returns TM_ENONFINITE / TM_ESTEP if any state
 * failed (the other states are still integrated). */
tm_status tm_run(tm_problem* p, tm_integrator integ, int64_t B, float* m, const float* Ha,
                 double* t, double* dt, int64_t* steps_out, const tm_run_cfg* cfg,
                 tm_run_stats* stats, hipStream_t stream);

/* ---- Field without allocation ------------------------------------------- */

/* Size of the fixed device scratch buffer of tm_demag_noalloc, per device. */
#define TM_NOALLOC_SCRATCH_BYTES (32ll << 20)

/* tm_demag without any device allocation, for callers that cannot allocate:
 * code under HIP graph capture, serving loops that must not reach the
 * allocator, harnesses that forbid it.  Same arguments, kernels and
 * summation order as tm_demag, so the result is bitwise tm_demag's.
 * Scratch (the padded state, 12 np B bytes with np = n rounded up to a
 * multiple of 128, and for PSYM6 / PSYM4 the slot sums, 384 ceil(n/32)^2 B
 * bytes) comes from one fixed library buffer of TM_NOALLOC_SCRATCH_BYTES per
 * device, set up by tm_init and kept until the process ends; no call here
 * allocates (the problem and its operator are made beforehand).
 * Operators: FP32 SYM6, BSR6, PSYM6, PSYM4 (TM_EINVAL for DENSE9 / FP64).
 * Errors: TM_EINVAL for bad arguments, an unsupported operator or a batch
 * whose scratch exceeds the buffer (the message gives both sizes), before
 * anything is enqueued; TM_EDEVICE on a HIP error.
 * Every call on one device shares that device's buffer: calls that overlap
 * in time on one device (other streams, other threads) race and must be
 * serialised by the caller; calls on one stream are ordered.  Stream-ordered,
 * returns after enqueueing. */
tm_status tm_demag_noalloc(tm_problem* p, int64_t B, const float* m, float* Hd, hipStream_t stream);

/* ---- Profiling ---------------------------------------------------------- */

/* Times the fused demag + effective-field + LL + stage-update kernel that
 * every Runge-Kutta stage of tm_run launches (the same kernel and launch
 * shape, on the problem's integration workspace for B states): `iters`
 * back-to-back launches between two HIP events recorded on `stream`.
 * Blocking.  avg_ms receives the mean duration of one launch; bytes_out
 * (may be NULL) the algorithmic bytes one launch moves (stored operator +
 * 24 bytes per tile and state).  The workspace contents are overwritten. */
tm_status tm_profile_field(tm_problem* p, int64_t B, int32_t iters, hipStream_t stream,
                           double* avg_ms, int64_t* bytes_out);

/* Same timing for one epilogue variant: mode 0 the stage update (as
 * tm_profile_field), 1 the demag field only, 2 the last Dormand-Prince stage
 * with its float64 error estimate, 3 the operator pass alone (for PSYM6 the
 * tile kernel without the reduction + epilogue launch; otherwise as 0), 4 the
 * stage update as inside an attempt, each launch reading the previous one's
 * output (for the batched DENSE9 product: the right operand the previous
 * stage wrote, no conversion pass; otherwise as 0). */
tm_status tm_profile_field_mode(tm_problem* p, int64_t B, int32_t mode, int32_t iters,
                                hipStream_t stream, double* avg_ms, int64_t* bytes_out);

/* Durations of the operator pass inside an integration: runs B states for
 * exactly cfg->max_attempts attempted steps (>= 1, <= 100000) as tm_run does
 * (same kernels, launch shapes and order; m, t and dt are updated the same
 * way; launched directly rather than from a captured graph), and stamps every
 * launch of the operator kernel -- the pair-symmetric tile pass, the fused
 * stage kernel of SYM6, the sparse kernel of BSR6 or the batched product of
 * DENSE9 -- with its own start and end (hipExtLaunchKernelGGL events on
 * `stream`).  The launches are queued behind a hold kernel (2 ms + 1 ms per
 * attempt, at most 200 ms) so that they run back to back as in a graph
 * replay.  op_ms receives the sum of those durations [ms], op_launches the
 * number of launches (DP45: 1 + 6 per attempt; RK4: 4 per step).  Blocking.
 * TM_EBUSY if called while another timing runs on the same thread;
 * otherwise the errors of tm_run. */
tm_status tm_profile_run(tm_problem* p, tm_integrator integ, int64_t B, float* m, const float* Ha, double* t,
                         double* dt, const tm_run_cfg* cfg, double* op_ms, int64_t* op_launches,
                         hipStream_t stream);

/* Number of launch shapes (workgroup width x target tiles per workgroup x
 * load kind) the fused field kernel is compiled for. */
int32_t tm_num_shapes(void);

/* Launch parameters of shape `shape`: workgroup threads, target tiles per
 * workgroup, nontemporal operator loads (0/1), waves-per-SIMD cap. */
tm_status tm_shape_info(int32_t shape, int32_t* threads, int32_t* tiles, int32_t* nontemporal,
                        int32_t* waves_cap);

/* Launch shape p's field kernel uses now (the default for its tile count
 * until tm_problem_set_shape or tm_problem_tune changes it). */
tm_status tm_problem_shape(const tm_problem* p, int32_t* shape);

/* Fixes the launch shape of p's field kernel (0 <= shape < tm_num_shapes(),
 * or -1 for the default chosen from the tile count).  The shape sets the
 * summation order of the demag product, so results are bitwise reproducible
 * for a fixed shape and independent of the batch size. */
tm_status tm_problem_set_shape(tm_problem* p, int32_t shape);

/* Autotuner: times every candidate (|iters| launches each, B states) and
 * keeps the fastest for p.  Blocking.  chosen / best_ms may be NULL.  For the
 * six-plane stage kernel (SYM6) the candidates are its launch shapes and
 * chosen is the shape kept.  For a DENSE9 operator in FP32 / BF16X3 / FP16X3
 * (the batched product) the candidates are the numbers of K splits (2, 3, 4,
 * 5, 6, 8) and, for a single layer of tiles (component-blocked operator),
 * the aligned work plans 100 + nq (K in nq super-ranges, nq = 2 .. 8 where
 * nq divides the z columns' chunk count and the z row blocks pair up), and
 * chosen is the choice kept; it sets the summation order, so results are
 * bitwise reproducible for a fixed choice and independent of the batch.  For PSYM6 / PSYM4 it times the evaluation with
 * cached (chosen = 0) and with nontemporal (chosen = 1) operator loads in the
 * tile pass and keeps the faster (the results are the same either way).  For
 * the other operators (one kernel shape each) it only times that kernel and
 * reports chosen = -1.
 * Every result is kept in a process-wide table keyed by (device architecture
 * and compute-unit count, layout, precision, tile count, B).  iters >= 1
 * reuses the table's result for p's key, if there is one, without timing
 * (best_ms is then the stored time); iters <= -1 always times (|iters|
 * launches per candidate) and replaces the entry.  iters = 0: TM_EINVAL. */
tm_status tm_problem_tune(tm_problem* p, int64_t B, int32_t iters, hipStream_t stream,
                          int32_t* chosen, double* best_ms);

/* Applies a choice as tm_problem_tune reports it, without timing: a launch
 * shape for SYM6, a K-split count or aligned plan for the batched DENSE9 product, 0 / 1
 * (cached / nontemporal operator loads) for PSYM6 / PSYM4.  For reproducing
 * a known configuration (a profiling run, another process) exactly.
 * TM_EINVAL if the choice is not a candidate for p (nothing changes then). */
tm_status tm_problem_apply(tm_problem* p, int32_t choice);

/* The autotuner's table as a JSON file (one entry per line: arch, cus,
 * layout, prec, n, batch, choice, ms), so that a later process reuses the
 * tuned choices.  tm_tune_cache_save writes every entry (TM_EINVAL if the
 * file cannot be written); tm_tune_cache_load merges the entries of a file
 * written by tm_tune_cache_save (TM_ENOTFOUND if it cannot be read, TM_EINVAL
 * if it is not such a file); tm_tune_cache_clear empties the table;
 * tm_tune_cache_size gives its number of entries.  An entry whose choice is
 * not a candidate for the problem it is looked up for is ignored. */
tm_status tm_tune_cache_save(const char* path);
tm_status tm_tune_cache_load(const char* path);
tm_status tm_tune_cache_clear(void);
tm_status tm_tune_cache_size(int64_t* entries);

/* ---- Serving: continuous batching of relaxation requests -------------- */

typedef struct {
    int64_t memory_budget;   /* bytes for tensors + slots (0: the context budget) */
    int32_t max_slots;       /* states per geometry group (batch width), >= 1 */
    int32_t max_groups;      /* geometry groups resident at once, >= 1 */
    int32_t steps_per_round; /* attempted steps per group between scheduler checks */
    tm_prec prec;            /* operator precision (FP32 only at present) */
    int32_t max_active;      /* groups advanced at once, those with the oldest requests
                                first (0: every resident group) */
} tm_server_cfg;

typedef struct {
    int64_t n;
    const double* centers;   /* host [n][3] */
    const double* sizes;     /* host [n][3] */
    tm_material mat;
    double Ha[3];            /* applied field [A/m] */
    const float* m0;         /* host [n][3] initial state */
    double dt0;              /* initial step [s] */
    double atol, rtol;
    double dmdt_stop;        /* equilibrium threshold on max_a |dm/dt|_a [1/s] */
    int64_t max_steps;       /* accepted-step cap */
} tm_request;

typedef struct {
    int32_t status;          /* TM_OK (equilibrium reached), TM_EBUSY (still running),
                                TM_ESTEP (step cap reached first, or step underflow),
                                TM_ENONFINITE, TM_ENOMEM (larger than the whole budget) */
    int64_t steps;           /* accepted steps */
    double t;                /* simulated time [s] */
    double latency_ms;       /* submit -> completion wall time */
    int32_t cache_hit;       /* 1 if the tensor came from the cache */
} tm_result;

/* Creates a server with its own scheduler thread on the context's device. */
tm_status tm_server_create(tm_ctx* ctx, const tm_server_cfg* cfg, tm_server** out);

/* Queues a request (host data copied).  Returns a ticket. */
tm_status tm_server_submit(tm_server* s, const tm_request* req, uint64_t* ticket);

/* Result of a ticket.  wait = 1 blocks until it completes.  If m_out is not
 * NULL (host [n][3]) the final state is copied there once complete. */
tm_status tm_server_poll(tm_server* s, uint64_t ticket, int32_t wait, tm_result* res, float* m_out);

/* Stops the scheduler after draining the queue, frees its memory. */
tm_status tm_server_destroy(tm_server* s);

#ifdef __cplusplus
}
#endif
#endif /* TILEMAG_H */
