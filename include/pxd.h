/*
 * pxd.h -- C ABI of the MI355X (gfx950) evaluator for pixelated multi-layer
 * MoM structures (arXiv 2412.17617).
 *
 * The library evaluates batches of candidate pixel maps: for every candidate
 * and every frequency it selects the active RWG functions, gathers their
 * rows and columns out of a precomputed parent impedance matrix (Eqs. 3-5),
 * solves the dense system Z I = V for every port (Eq. 2), forms the
 * S-parameters (Eqs. 6-7) and reduces them to the figure of merit of
 * Eqs. 8-9.  A native host routine builds the structure (mesh, basis-function
 * classification of Section II-C) and fills the parent matrices.
 *
 * Conventions shared by every entry point:
 *  - Return value: PXD_OK (0) or a negative PXD_E* code.  Nothing throws
 *    across the ABI.  pxd_last_error() returns a message for the last failure
 *    on a context (or on the thread, for calls that take no context).
 *  - Complex numbers are interleaved (re, im) doubles (complex128) or floats.
 *  - Matrices are row-major; parent matrices are symmetric so row and column
 *    order coincide.
 *  - Host pointers passed in are only read during the call; the library
 *    copies what it keeps.  Output host buffers are owned by the caller.
 *  - *_device entry points take device pointers (for example memory owned by
 *    PyTorch) and a hipStream_t passed as void* (NULL = HIP's default
 *    stream); work is ordered on that
 *    stream and the call returns without synchronising it.  Device buffers
 *    are borrowed only for the duration of the call.
 *  - Units are SI: metre, hertz, ohm.
 *  - One context must not be used from two host threads at once.
 */
#ifndef PXD_H
#define PXD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PXD_OK 0
#define PXD_EINVAL (-1)     /* bad argument (null pointer, size out of range) */
#define PXD_ENOMEM (-2)     /* host or device allocation failed */
#define PXD_ENOTLOADED (-3) /* parent matrices, map or FoM table not loaded */
#define PXD_EDEVICE (-4)    /* HIP runtime error */
#define PXD_ESHAPE (-5)     /* inconsistent sizes between loaded objects */

/* Basis-function classes (Section II-C, Fig. 2(a)); a function is active iff
 * every cell it references (cell_a, cell_b; -1 = none) is on. */
#define PXD_KIND_ALWAYS 0  /* feed and port functions */
#define PXD_KIND_INNER 1   /* inside one pixel */
#define PXD_KIND_INTER 2   /* between two side-adjacent pixels */
#define PXD_KIND_PIXPORT 3 /* between a feed and its adjacent pixel */
#define PXD_KIND_VIA 4     /* vertical strip joining layers 0 and 1 */

/* Per-item status codes written by the evaluator. */
#define PXD_STATUS_OK 0
#define PXD_STATUS_FALLBACK 1     /* mixed precision did not converge; FP64 result returned */
#define PXD_STATUS_NONFINITE (-1) /* a non-finite value reached S */
#define PXD_STATUS_SINGULAR (-2)  /* an exactly zero pivot was met */
#define PXD_STATUS_SIZE (-3)      /* active size above the bound a captured graph was built for (or < P);
                                     the item's S entries are NaN */
/* A candidate whose worst item status is negative has no valid S at some
 * frequency: its FoM is +inf and it is never the argmin (Algorithm 1 accepts
 * only a strict improvement of a valid FoM).  The argmin is -1 when no
 * candidate of the batch has a finite FoM. */

/* Order in which the persistent workgroups take (candidate, frequency) items. */
#define PXD_SCHED_AUTO 0       /* tuned value if the context has one, else frequency-major */
#define PXD_SCHED_FREQ_MAJOR 1 /* all candidates of one frequency (largest first), then the next frequency */
#define PXD_SCHED_SIZE_MAJOR 2 /* all frequencies of the largest candidate first (uneven batches) */

/* Arithmetic of the dense solve. */
#define PXD_PREC_FP64 0    /* complex128 LU, no refinement ("plain") */
#define PXD_PREC_MIXED32 1 /* complex64 LU + FP64 residual and iterative refinement */
#define PXD_PREC_MIXED_BF16 2 /* as MIXED32, the rank-64 block-column updates on BF16 operands (FP32 accumulation) */
#define PXD_PREC_MIXED_F16 3  /* as MIXED32, the rank-64 block-column updates on FP16 operands (FP32 accumulation) */
/* as MIXED32, the trailing updates on split BF16 operands: x = hi + lo (both BF16), each real product as
 * hi*hi + hi*lo + lo*hi on the BF16 MFMA with FP32 accumulation (~2^-16 relative, FP32's exponent range);
 * tiled LU.  The plain BF16 and FP16 modes run on the persistent LU only (active sizes up to 2,048). */
#define PXD_PREC_MIXED_BF16X3 4

/* ---------------------------------------------------------------- structure */

/* Workload geometry.  Layer l lies in z = -l*h; pixel (l, x, y) covers
 * [x a, (x+1) a] x [y a, (y+1) a].  Each pixel carries two triangles with
 * checkerboard-alternating diagonals.  Port k sits at the middle cell of grid
 * side port_side[k] (0 right, 1 top, 2 left, 3 bottom) on layer port_layer[k].
 * Via v joins cell (0, via_x[v], via_y[v]) and cell (1, ...), hanging under
 * the cell's lower side. */
typedef struct pxd_geometry {
  int32_t n_layers, nx, ny;
  double a, h;
  double eps_r, tan_d; /* homogeneous medium: eps = eps0 eps_r (1 - j tan_d) */
  int32_t n_ports;
  const int32_t* port_side;
  const int32_t* port_layer;
  int32_t n_vias;
  const int32_t* via_x;
  const int32_t* via_y;
  int32_t sub;         /* squares per pixel side (0 or 1: 2 triangles per pixel; 2: 8; 3: 18), each square
                          split into two right triangles, diagonals alternating over the squares
                          (the mesh study of Section V); feeds attach to square sub / 2 of their side */
} pxd_geometry;

typedef struct pxd_problem pxd_problem;

/* Build mesh and RWG functions in canonical order: inner (cell order; within
 * a pixel by the edge's midpoint, y first), inter-pixel horizontal then
 * vertical (each pixel pair's squares in order along the side), pixel-port,
 * via (per via: top junctions, then diagonals and sub-strip sides, then
 * bottom junctions, each by position), feed diagonals, port edges last (port
 * order).  *out is owned by the caller (pxd_problem_destroy). */
int pxd_problem_create(const pxd_geometry* g, pxd_problem** out);
void pxd_problem_destroy(pxd_problem* p);
/* Parent size M, cell count and port count. */
int pxd_problem_sizes(const pxd_problem* p, int32_t* M, int32_t* n_cells, int32_t* n_ports);
/* Classification arrays (length M each; port arrays length n_ports):
 * kind, cell_a, cell_b, the parent index of each port's delta-gap function
 * and its edge length.  Any pointer may be NULL to skip that array. */
int pxd_problem_classification(const pxd_problem* p, uint8_t* kind, int32_t* cell_a, int32_t* cell_b,
                               int32_t* port_bf, double* port_len);
/* Fill the parent impedance matrices of the EFIE (Eqs. 1-2), mixed-potential
 * Galerkin with RWG functions, kernel exp(-jkR)/(4 pi R), 4-point triangle
 * rule, closed-form 1/R extraction on near pairs; upper triangle computed and
 * mirrored.  Z_out: F x M x M complex128, row-major, caller-owned (host).
 * n_threads <= 0 uses every hardware thread.  Host only; needs no GPU. */
int pxd_problem_fill(const pxd_problem* p, int32_t F, const double* freqs_hz, double* Z_out, int32_t n_threads);
/* The same fill on GPU `device` (Section II-A's parent fill, the paper's
 * Phase 2, run on the GPU instead of host cores): one FP64 thread per
 * (test triangle, source triangle, test point) builds the source integrals,
 * one per (m, n >= m) assembles Z_mn and mirrors it.  Z_out: device pointer,
 * F x M x M complex128, caller-owned; work is enqueued on `stream` (a
 * hipStream_t, NULL = default) and finished when the call returns.  Allocates
 * a temporary table of T x T x 256 bytes (T triangles) plus the geometry;
 * PXD_ENOMEM if that fails.  Agrees with pxd_problem_fill up to the rounding
 * of the device math library. */
int pxd_problem_fill_device(const pxd_problem* p, int32_t device, void* stream, int32_t F, const double* freqs_hz,
                            double* Z_out);

/* ---------------------------------------------------------------- evaluator */

typedef struct pxd_options {
  int32_t device;          /* HIP device ordinal */
  int32_t precision;       /* PXD_PREC_* */
  int32_t ir_max_iter;     /* refinement iterations before FP64 fallback (default 10) */
  double ir_tol;           /* relative accuracy of every S entry at which refinement stops (default 1e-7):
                              the error left after a step is estimated as rho / (1 - rho) times the largest
                              change the step made to any S entry, rho the observed contraction (ratio of the last two
                              largest changes, so at least two steps are taken), and must be below
                              ir_tol |S_ij| + 1e-11 */
  int32_t wg_per_cu;       /* persistent workgroups per compute unit: 1 or 2 (0 = tuned, else 2) */
  int32_t half_subpanel;   /* register sub-panel of the LU: 1 full width, 2 half width (0 = tuned, else full) */
  int32_t schedule;        /* PXD_SCHED_* */
  int32_t lu_path;         /* PXD_PATH_*: which dense LU solves the items */
  int32_t tile_kb;         /* tiled path: block-column width 64 or 128 (0 = tuned, else 128) */
  int32_t tile_shape;      /* tiled path: output tile of the trailing update, 1 = 128 x 64 (four waves, two
                              workgroups per CU), 2 = 64 x 64 (four waves, three per CU), 3 = 128 x 64 (eight
                              waves, two per CU), 4 = 128 x 128 (eight waves, one per CU); 3 and 4 are FP64 and
                              FP32 updates only (the split-BF16 update takes 1 for them); 0 = tuned, else 2 */
  double ws_gib;           /* tiled path: workspace cap in GiB (0 = 80 % of the free device memory,
                              at most 64 GiB); fixes how many items are factored together */
  int32_t refine;          /* tiled path, mixed modes: PXD_REFINE_* */
} pxd_options;

/* Refinement of the tiled path's mixed modes.  Per item: each item's FP64
 * residuals re-gather its rows of Z_A from the complex128 parent.  Lock step:
 * the items of one frequency refine together, their residuals one product
 * Z_f[U, U] X over the union U of the call's active sets (one pass over the
 * parent rows per frequency and step); the stop test and the solves are the
 * same, so the results agree up to the residuals' summation order.  Auto:
 * lock step when |U| is at most 1.25 times the largest active size. */
#define PXD_REFINE_AUTO 0
#define PXD_REFINE_PER_ITEM 1
#define PXD_REFINE_LOCKSTEP 2

/* Dense LU of the evaluation (Eq. 2).  Persistent: one workgroup per item,
 * the whole factorisation and solve in one persistent launch over all items
 * (active sizes up to 2,048).  Tiled: the items are factored in chunks, in
 * lock step, one launch per step of each block column with many workgroups
 * per item (a panel kernel per item, then the interchanges and U12 solve and
 * the trailing-matrix update tiled over the item's columns / output tiles);
 * active sizes up to 10,240 in FP64 and up to 5,696 (P = 3) in the mixed
 * modes, whose solves keep the right-hand sides in LDS; not available in
 * graphs or the no-allocation
 * entry point. */
#define PXD_PATH_AUTO 0       /* tuned value for the size class, else persistent up to 2,048 and tiled above */
#define PXD_PATH_PERSISTENT 1
#define PXD_PATH_TILED 2

typedef struct pxd_ctx pxd_ctx;

/* A FoM term (Eq. 9 in closed form): value = 10^log10_factor * |S_ij|^power,
 * summed over the frequencies whose band equals `band`.  i, j are 0-based. */
typedef struct pxd_fom_term {
  int32_t band;
  int32_t i, j;
  double log10_factor;
  double power;
} pxd_fom_term;

typedef struct pxd_stats {
  int64_t items;          /* (candidate, frequency) solves in the last call */
  int64_t fallbacks;      /* items re-solved in FP64 after refinement failed */
  int64_t ir_iterations;  /* refinement iterations summed over items */
  int32_t max_active;     /* largest active size N in the last call */
  int32_t min_active;
  double ms_expand, ms_solve, ms_fallback, ms_fom; /* stage times of the last call (events) */
  double ms_base_inverse; /* low-rank calls: time of the base-map inverse (0 if reused) */
  int32_t base_reused;    /* low-rank calls: 1 if the cached base inverse served the call */
  int32_t update_launches; /* tiled path with profiling on: trailing-update launches of the last call */
  double ms_update;       /* ... their summed duration (an event pair around each launch) */
  double update_gflop;    /* ... their algorithmic work: 8 kb (N - Kend)(ncols - Kend) real flops per item
                             and block column (complex multiply-add = 8 flops) */
  double update_gbyte;    /* ... and their algorithmic memory traffic: the trailing block read and written
                             once, L21 and U12 read once (bytes per complex entry 8 or 16) */
} pxd_stats;

int pxd_create(const pxd_options* opt, pxd_ctx** out);
void pxd_destroy(pxd_ctx* ctx);
const char* pxd_last_error(const pxd_ctx* ctx); /* ctx may be NULL: thread-local last error */

/* Parent matrices: F x M x M complex128 row-major host array, frequencies in Hz.
 * The library keeps a device copy and, in the mixed modes, a complex64 copy
 * when that fits beside it with 8 GiB of device memory to spare; without the
 * copy the mixed modes round the complex128 parent as they gather and use the
 * tiled LU. */
int pxd_load_parent(pxd_ctx* ctx, int32_t M, int32_t F, const double* freqs_hz, const double* Z);
/* Same, with the parent filled on the context's device by
 * pxd_problem_fill_device straight into the context's copy (no host matrix). */
int pxd_load_parent_problem(pxd_ctx* ctx, const pxd_problem* p, int32_t F, const double* freqs_hz);

/* Pixel-to-RWG map (Section II-C): per parent function its kind and the cells
 * it needs (cell_b = -1 if one); P ports with their parent function index
 * (ports must be the last P functions, in port order) and edge length; Z0. */
int pxd_load_map(pxd_ctx* ctx, int32_t n_cells, int32_t M, const uint8_t* kind, const int32_t* cell_a,
                 const int32_t* cell_b, int32_t P, const int32_t* port_bf, const double* port_len, double z0);

/* FoM table and per-frequency band id (-1 = no band). */
int pxd_set_fom(pxd_ctx* ctx, int32_t n_terms, const pxd_fom_term* terms, const int8_t* band_of_freq);
/* The FoM of Eqs. 8-9 with the Section III-B bands (p1 = [5.15, 5.925] GHz,
 * p2 = [6.425, 7.125] GHz, f_i between them, f_s = the rest of [3, 9] GHz);
 * terms whose S entry exceeds the port count are dropped. */
int pxd_set_fom_paper(pxd_ctx* ctx);

/* FoM variants of Section III-D, as alternative term tables (bands as above). */
#define PXD_FOM_PAPER 0 /* Eqs. 8-9 */
#define PXD_FOM_REJ 1   /* rw_s1, rw_s2 replaced by 10^((-S_dB - 45) / 10) */
#define PXD_FOM_ISO 2   /* Eqs. 8-9 plus 1/rw_oi^iso = 1 / 10^((-S32_dB - 35) / 15) over p1 and p2 */
int pxd_set_fom_variant(pxd_ctx* ctx, int32_t variant);

/* Evaluate candidates given as flips of a base map: candidate c toggles cells
 * cells[offsets[c] .. offsets[c+1]).  Outputs (host, caller-owned, any may be
 * NULL): S_out n_cand x F x P x P complex128; fom_out n_cand (+inf for a
 * candidate with a negative status); status n_cand (worst item status);
 * argmin_out the lowest-index minimum-FoM candidate among those with a finite
 * FoM, -1 if there is none (Algorithm 1's arg min over the evaluated leaves). */
int pxd_evaluate_flips(pxd_ctx* ctx, const uint8_t* base_map, int32_t n_cand, const int32_t* offsets,
                       const int32_t* cells, double* S_out, double* fom_out, int32_t* status,
                       int32_t* argmin_out);

/* Same with device pointers on `stream` (a hipStream_t); n_flips is the
 * length of `cells`.  argmin_out is a device int32. */
int pxd_evaluate_flips_device(pxd_ctx* ctx, void* stream, const uint8_t* base_map, int32_t n_cand,
                              const int32_t* offsets, const int32_t* cells, int32_t n_flips, double* S_out,
                              double* fom_out, int32_t* status, int32_t* argmin_out);

/* For callers that cannot allocate device memory (code between allocation-free
 * points of a serving loop, harnesses that forbid hipMalloc): the same
 * evaluation as pxd_evaluate_flips_device, with the same arguments, outputs
 * and stream semantics, but every buffer the kernels need beyond the caller's
 * inputs and outputs (active lists, item order, counters, per-item status,
 * the FP64 hand-off list and the LU workspace slots) is carved out of a
 * static device array of 64 MiB that each GPU holds from library load to
 * process end.  No hipMalloc, hipFree or other allocating routine is called;
 * the call reads back two integers (the batch's smallest and largest active
 * size) and so synchronises `stream` once.  It runs as many persistent
 * workgroups as workspace slots fit (at least one).  A batch whose active
 * lists (n_cand x (M + 2) int32 plus n_cand x F int32, twice that in the mixed
 * modes) plus one slot do not fit is refused with PXD_ESHAPE and a message
 * giving the sizes.  Every call on one GPU shares that array and leaves its
 * contents behind (counters are cleared at the start of each call): calls
 * that overlap on one GPU, from any context or thread, race and must not be
 * made.  The context must be loaded (parent, map, FoM) as for the other
 * entry points; loading allocates, this call does not. */
int pxd_evaluate_flips_device_noalloc(pxd_ctx* ctx, void* stream, const uint8_t* base_map, int32_t n_cand,
                                      const int32_t* offsets, const int32_t* cells, int32_t n_flips, double* S_out,
                                      double* fom_out, int32_t* status, int32_t* argmin_out);

/* Flip candidates evaluated from the inverse of the base map instead of one
 * dense factorisation each (a variant the paper does not use; it gives the
 * S of Eqs. 6-7 for the candidate's Z_A of Eq. 5 up to rounding).  With
 * G = Z_B^-1 for the base active set (port loads included), a candidate that
 * drops the base functions R and adds the functions E is solved by block
 * elimination: the removed functions by the Schur-complement identity for the
 * inverse of a principal submatrix, the added ones by the block inverse of the
 * bordered matrix.  Cost per (candidate, frequency): one pass over G per four
 * added functions plus O((|R| + |E|)^3), against O(N^3) for a dense solve.
 * G is computed in FP64 (F x N_B x N_B complex128 on the device) on the first
 * call for a base map and reused while the base map, the parent and the map
 * stay the same.  Candidates that drop more than 16 or add more than 8 base
 * functions, relative to the base map, are solved by the dense FP64 path in the
 * same call, whatever the context's precision (counted in pxd_stats.fallbacks).
 * Z must be complex symmetric (Galerkin EFIE), which the identities use.
 * Arguments, outputs and errors as for pxd_evaluate_flips; item status
 * SINGULAR if the base matrix or one of the small blocks has a zero pivot. */
int pxd_evaluate_flips_lowrank(pxd_ctx* ctx, const uint8_t* base_map, int32_t n_cand, const int32_t* offsets,
                               const int32_t* cells, double* S_out, double* fom_out, int32_t* status,
                               int32_t* argmin_out);

/* Row a1 alone: active index sets (Eq. 3) of each candidate.  N_out n_cand;
 * idx_out n_cand x M (row c holds N_out[c] ascending indices).  Host buffers. */
int pxd_expand(pxd_ctx* ctx, const uint8_t* base_map, int32_t n_cand, const int32_t* offsets,
               const int32_t* cells, int32_t* N_out, int32_t* idx_out);

/* Row a2 alone: the gathered matrix Z_parent(f)[I, I] (Eq. 5) for index set
 * idx (N ascending parent indices) at frequency index f.  ZA_out: N x N
 * complex128 host buffer. */
int pxd_gather(pxd_ctx* ctx, int32_t f, int32_t N, const int32_t* idx, double* ZA_out);

int pxd_get_stats(const pxd_ctx* ctx, pxd_stats* out);
/* Profiling of the tiled path: when on, every trailing-update launch is
 * bracketed by a pair of HIP events on the call's stream and its algorithmic
 * work is counted (pxd_stats.update_*); off by default. */
int pxd_set_profiling(pxd_ctx* ctx, int32_t on);

/* The verdict the mixed-precision kernels take after refinement step `iters`
 * (1-based) of an item, exposed so that the rule can be checked on the host.
 * m: the largest change of any S_ij (Eq. 6) the step makes; m_prev: that of
 * the previous step (0 before the first); target: min over the entries of
 * ir_tol |S_ij| + 1e-11.  With the observed contraction rho = m / m_prev (1 on
 * the first step) the error left in every entry is bounded by
 * m rho / (1 - rho).  Returns 1 (converged: that bound is below target and
 * rho < 0.9), 2 (give up from the third step on: rho >= 1, a NaN, or more
 * steps needed than ir_max allows; the item goes to the FP64 path) or 0 (take
 * another step); PXD_EINVAL if iters or ir_max is below 1.  Needs no GPU. */
int pxd_refine_verdict(int32_t iters, int32_t ir_max, double m, double m_prev, double target);

/* Candidates given as whole maps (an uneven batch: any mix of active sizes in
 * one persistent launch): maps is n_maps x n_cells, row c = candidate c.
 * Outputs as for pxd_evaluate_flips.  Host buffers. */
int pxd_evaluate_maps(pxd_ctx* ctx, int32_t n_maps, const uint8_t* maps, double* S_out, double* fom_out,
                      int32_t* status, int32_t* argmin_out);
/* Same with device pointers on `stream`. */
int pxd_evaluate_maps_device(pxd_ctx* ctx, void* stream, int32_t n_maps, const uint8_t* maps, double* S_out,
                             double* fom_out, int32_t* status, int32_t* argmin_out);

/* ------------------------------------------------------------ autotuning */

/* One configuration tried by pxd_autotune and its measured evaluator time. */
typedef struct pxd_tune_entry {
  int32_t rows_per_thread; /* size class Q: active sizes up to 256 Q (Q = 1, 2, 4, 8, 16) */
  int32_t wg_per_cu, half_subpanel, schedule; /* persistent path (wg_per_cu, half_subpanel 0 for tiled) */
  int32_t lu_path;         /* PXD_PATH_PERSISTENT or PXD_PATH_TILED */
  int32_t tile_kb;         /* tiled path: block-column width */
  int32_t tile_shape;      /* tiled path: trailing-update output tile (1 = 128 x 64, 2 = 64 x 64) */
  int32_t reserved;
  double ms;               /* evaluator time (solve + fallback), best of n_reps */
} pxd_tune_entry;

/* Time every configuration on this batch (host buffers, as
 * pxd_evaluate_flips), n_reps times each, and keep the fastest for the
 * batch's precision and size class; later calls whose options say "tuned"
 * use it.  Configurations: the persistent path (active sizes up to 2,048;
 * workgroups per CU 1 or 2 x register sub-panel full or half width x item
 * order) and the tiled path (block columns of 64 or 128 x output tiles of
 * 128 x 64 or 64 x 64 x item order).  A choice the context's options fix
 * (lu_path, tile_kb 64/128, tile_shape 1/2, wg_per_cu > 0, half_subpanel 1
 * or 2, schedule not AUTO) is not searched.  report (may be
 * NULL) receives up to max_report entries, *n_report the number written; the
 * chosen one is report[0]. */
int pxd_autotune(pxd_ctx* ctx, const uint8_t* base_map, int32_t n_cand, const int32_t* offsets,
                 const int32_t* cells, int32_t n_reps, pxd_tune_entry* report, int32_t max_report,
                 int32_t* n_report);
/* Tuned table as text (one line per precision and size class), and back. */
int pxd_tune_save(const pxd_ctx* ctx, const char* path);
int pxd_tune_load(pxd_ctx* ctx, const char* path);

/* ------------------------------------------------------------ HIP graphs */

typedef struct pxd_graph pxd_graph;

/* Capture the whole device-side evaluation of a batch (expand, order,
 * evaluator, fallback, FoM, argmin) into a HIP graph.  All pointers are
 * device pointers that must stay valid while the graph exists; the graph
 * reads their contents at each launch, so the caller may change the map or
 * flips in place between launches.  base_stride must be 0: one base map plus
 * flips (offsets/cells as in pxd_evaluate_flips_device); whole-map batches
 * (base_stride = n_cells) are refused with PXD_EINVAL.  Nothing in the captured
 * work synchronises with the host, so the launch is sized for active sizes
 * up to n_max_active: an item above it gets PXD_STATUS_SIZE.  The graph owns
 * its own workspace (allocated here), so it does not disturb other calls on
 * the context; the context must outlive it. */
int pxd_graph_create(pxd_ctx* ctx, const uint8_t* base_map, int64_t base_stride, int32_t n_cand,
                     const int32_t* offsets, const int32_t* cells, int32_t n_max_active, double* S_out,
                     double* fom_out, int32_t* status, int32_t* argmin_out, pxd_graph** out);
/* Launch the captured evaluation on `stream` (NULL = HIP's default stream). */
int pxd_graph_launch(pxd_graph* g, void* stream);
void pxd_graph_destroy(pxd_graph* g);

/* ------------------------------------------------------------ CNN surrogate
 *
 * A small convolutional network that predicts, from a pixel map and a
 * frequency, the S entries the FoM of Eqs. 8-9 weighs most, so that a search
 * step of Algorithm 1 can rank every candidate and solve only the best k
 * exactly (the exact solve remains the judge of every accepted flip).  It is
 * not part of the paper's method.  Architecture (all kernels hand-written):
 *   x0   = map as an image (channels = layers; cell l*ny*nx + y*nx + x)
 *   a1   = relu(conv3x3(x0)),  a2 = pool2(relu(conv3x3(a1))),
 *   a3   = relu(conv3x3(a2)),  a4 = pool2(relu(conv3x3(a3)))
 *   h    = relu(flatten(a4) Wf + e(u) We + bh),  out = h Wo + bo
 * conv3x3: zero padding 1, weights [tap = 3 dy + dx][c_in][c_out] applied to
 * x[y + dy - 1][x + dx - 1]; pool2: 2 x 2 mean, odd last row/column dropped;
 * flatten order (y, x, channel); e(u)_{2j} = sin((j+1) pi u),
 * e(u)_{2j+1} = cos((j+1) pi u), u = (f - f_lo) / (f_hi - f_lo).
 * Outputs per (map, frequency) and predicted entry, in entry order: ln|S|
 * and the unit phasor (cos arg S, sin arg S), so S = |S| (cos + j sin); the
 * squared error on ln|S| weighs relative error alike for large and tiny
 * entries, as the FoM's powers of |S| do.  Parameters: one float32 vector, tensors in the order W1 b1 W2 b2 W3
 * b3 W4 b4 Wf We bh Wo bo, each row-major in the shapes above.
 * The products run on MFMA: FP32 (16x16x4) or BF16 operands with FP32
 * accumulation (16x16x16); parameters, activations and gradients are kept in
 * FP32.  Loss: mean squared error over all outputs.  Optimiser: AdamW with
 * bias-corrected moments, decay on every parameter. */

#define PXD_SUR_FP32 0
#define PXD_SUR_BF16 1

/* Inference path of pxd_sur_forward and pxd_sur_rank (training always uses
 * the generic products).  FUSED: the four convolutions of one map run in one
 * workgroup with BF16 activations held in LDS, and the head's output layer
 * forms its hidden activations in registers; BF16 only, ny and nx multiples
 * of 8, n_layers <= 8, channels each 32 or 64, hidden a power of two
 * >= 32.  Same operand rounding as the generic BF16 products, FP32 sums in
 * another order.  AUTO takes FUSED where it applies, else GENERIC. */
#define PXD_SUR_INFER_AUTO 0
#define PXD_SUR_INFER_GENERIC 1
#define PXD_SUR_INFER_FUSED 2

typedef struct pxd_sur_config {
  int32_t device;
  int32_t n_layers, ny, nx;  /* map shape */
  int32_t channels[4];       /* conv widths (e.g. 32 32 64 64), each <= 256 */
  int32_t hidden, emb;       /* head width; frequency embedding size (even) */
  int32_t n_entries;         /* predicted S entries, 1..4: (entry_i[k], entry_j[k]), 0-based */
  int32_t entry_i[4], entry_j[4];
  int32_t precision;         /* PXD_SUR_* */
  int32_t max_batch;         /* largest number of maps per call */
  int32_t inference;         /* PXD_SUR_INFER_*; FUSED where it does not apply gives PXD_EINVAL */
} pxd_sur_config;

typedef struct pxd_adamw {
  double lr, beta1, beta2, eps, weight_decay;
} pxd_adamw;

typedef struct pxd_sur pxd_sur;

/* freqs_hz: the F frequencies every map is evaluated at; f_lo, f_hi set u. */
int pxd_sur_create(const pxd_sur_config* cfg, int32_t F, const double* freqs_hz, double f_lo, double f_hi,
                   pxd_sur** out);
void pxd_sur_destroy(pxd_sur* s);
const char* pxd_sur_last_error(const pxd_sur* s);
int pxd_sur_num_params(const pxd_sur* s, int64_t* n);
/* The inference path in use: PXD_SUR_INFER_GENERIC or PXD_SUR_INFER_FUSED. */
int pxd_sur_inference_path(const pxd_sur* s, int32_t* path);
/* Uniform initialisation from SplitMix64(seed * 1000 + tensor index): weights
 * in +-sqrt(3 / fan_in) (fan_in = product of all but the last dimension),
 * biases in +-0.05.  Resets the optimiser state. */
int pxd_sur_init_params(pxd_sur* s, uint64_t seed);
/* Host float32 vectors of length num_params. set resets the optimiser state. */
int pxd_sur_set_params(pxd_sur* s, const float* params, int64_t n);
int pxd_sur_get_params(const pxd_sur* s, float* params, int64_t n);
/* Device pointers on `stream`: maps B x n_cells uint8 (0/1); out and target
 * B x F x (3 n_entries) float32. */
int pxd_sur_forward(pxd_sur* s, void* stream, int32_t B, const uint8_t* maps, float* out);
/* Loss (device float, may be NULL) and its gradient (device float32
 * num_params, may be NULL: kept inside) without updating the parameters. */
int pxd_sur_gradient(pxd_sur* s, void* stream, int32_t B, const uint8_t* maps, const float* target, float* grad,
                     float* loss);
/* Gradient then one AdamW step. */
int pxd_sur_train_step(pxd_sur* s, void* stream, int32_t B, const uint8_t* maps, const float* target,
                       const pxd_adamw* hp, float* loss);
/* Rank candidates (base map + CSR flips, device pointers as in
 * pxd_evaluate_flips_device) by the FoM of the predicted |S| = exp(ln|S|),
 * using the FoM table of `ctx` (terms on entries the network does not
 * predict are left out).  fom_pred: n_cand doubles (device); top: the k lowest, best first,
 * ties to the lower index (device int32). */
int pxd_sur_rank(pxd_sur* s, const pxd_ctx* ctx, void* stream, const uint8_t* base_map, int32_t n_cand,
                 const int32_t* offsets, const int32_t* cells, int32_t k, double* fom_pred, int32_t* top);
/* Training targets from exact S on the device: S is n x F x P x P complex128
 * (interleaved, the evaluator's S layout); target n x F x (3 n_entries)
 * float32: per predicted entry ln max(|S_ij|, 1e-30), cos arg S_ij,
 * sin arg S_ij (the outputs above).  Device pointers on `stream`; entries
 * beyond P give PXD_ESHAPE. */
int pxd_sur_encode(pxd_sur* s, void* stream, int32_t n, const double* S, int32_t P, float* target);

#ifdef __cplusplus
}
#endif
#endif /* PXD_H */
