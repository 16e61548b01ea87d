/* ldgmg.h -- C-ABI of the MI355X multigrid library for high-order LDG systems.
 *
 * The library solves A_h x_h = b_h, the linear system of a local discontinuous
 * Galerkin (LDG) discretisation on a uniform n^d Cartesian grid of the unit box
 * (paper: Saye, "A comparative study of efficient multigrid solvers for
 * high-order local discontinuous Galerkin methods", arXiv:2412.12506):
 *   - scalar elliptic (interface) problems, Section 2.1:
 *       A = sum_k G_k^T M_mu G_k + E;
 *   - Stokes saddle-point problems, Section 3.1, eq:components.
 * with the multigrid V-cycle of Algorithm 1 (block Jacobi, multi-coloured
 * block Gauss-Seidel or balanced block SAI smoothers, Section 2.3 and 3.3) as
 * the preconditioner of CG or left-preconditioned GMRES (Section 2.2).
 *
 * Conventions shared by every entry point
 *   - Elements are numbered lexicographically with x fastest:
 *       e = ix + n*iy + n*n*iz.
 *   - Vectors are element-major: v[e*bs + a].  Inside an element the scalar
 *     coefficients are ordered with the x-degree fastest; Stokes elements hold
 *     [u_1 .. u_d, p], each a block of (p+1)^d coefficients, so bs = (d+1)(p+1)^d.
 *   - "dev" pointers are device (HIP) memory owned by the caller; "host"
 *     pointers are host memory owned by the caller.  The library never keeps a
 *     caller pointer after a call returns.
 *   - `stream` is a hipStream_t passed as void*; NULL means the null stream.
 *     Work is enqueued on that stream; calls that must return host values
 *     (ldgmg_solve) synchronise that stream only.
 *   - Every function returns an int status (LDGMG_OK = 0, negative on error)
 *     and never throws across the ABI; ldgmg_last_error() gives a message
 *     (per calling thread).
 *   - A handle is not safe for concurrent use: calls on one handle must be
 *     serialised by the caller (they share the handle's device workspace).
 */
#ifndef LDGMG_H
#define LDGMG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  LDGMG_OK = 0,
  LDGMG_EINVAL = -1,    /* invalid argument (shape, option, NaN/Inf input)    */
  LDGMG_ENOMEM = -2,    /* over the HBM budget or device allocation failed    */
  LDGMG_EHIP = -3,      /* HIP runtime error                                  */
  LDGMG_ENOCONV = -4,   /* maxit reached; the info struct is still filled     */
  LDGMG_ESINGULAR = -5, /* rank-deficient local problem in the setup, or an
                           inconsistent right-hand side (ldgmg_rhs_check)     */
  LDGMG_ESTATE = -6     /* call not valid in the handle's state (e.g. no device data) */
};

enum { LDGMG_POISSON = 0, LDGMG_STOKES = 1 };
enum { LDGMG_BASIS_LEGENDRE = 0, LDGMG_BASIS_GL_NODAL = 1 };
enum { LDGMG_BC_DIRICHLET = 0, LDGMG_BC_NEUMANN = 1, LDGMG_BC_PERIODIC = 2 };
enum { LDGMG_SMOOTH_JACOBI = 0, LDGMG_SMOOTH_GS = 1, LDGMG_SMOOTH_SAI = 2 };
/* pre/post ordering (Section 2.4): first letter pre-smoother, second post;
 * O = forward (eq:B1 / colours in order), I = reverse (eq:BT / colours reversed) */
enum { LDGMG_ORDER_OO = 0, LDGMG_ORDER_OI = 1, LDGMG_ORDER_IO = 2, LDGMG_ORDER_II = 3 };
/* storage precision of the V-cycle's matrices (A on every level, the smoother
 * matrix B or D^-1): FP64, FP32, or LDGMG_BF16S = FP32 operators with the SAI
 * matrices B and B^T in BF16 (round to nearest even via FP32; SAI smoothers
 * only, EINVAL otherwise).  V-cycle vectors, transfers and all arithmetic are
 * FP64 in every mode (stored blocks are widened exactly as they are read); the
 * outer Krylov iteration, its FP64 operator and inner products are FP64. */
enum { LDGMG_FP64 = 0, LDGMG_FP32 = 1, LDGMG_BF16S = 2 };
/* device storage of the block-sparse matrices.  EXPANDED: every slot holds its
 * block.  POOLED: the distinct blocks of a matrix are stored once and every
 * slot holds a 4-byte block id; the setup builds each matrix as such a pool
 * (identical blocks are computed once), so both storages hold the same values
 * and give bitwise-equal results.  TILED: POOLED plus, for matrices with at
 * most 64 distinct column offsets (column - row), a [row][offset] table of
 * block ids and a copy of the pool in the operand layout of the FP64 matrix
 * cores: forward products then run as 16-row tiles of FP64 MFMA (same values,
 * FP64 products and sums, a different summation order).  AUTO: per matrix and
 * level, TILED (or POOLED beyond 64 offsets) when its distinct blocks take at
 * most 64 MiB and at most a quarter of the expanded bytes, else EXPANDED.
 * Pooled and tiled storage need a block size with a wave-mapped kernel (4, 8,
 * 9, 12, 16, 25, 27, 32, 36, 48, 64); other sizes are always expanded. */
enum { LDGMG_STORE_AUTO = 0, LDGMG_STORE_EXPANDED = 1, LDGMG_STORE_POOLED = 2, LDGMG_STORE_TILED = 3 };
enum { LDGMG_CG = 0, LDGMG_GMRES = 1 };

typedef struct ldgmg_hier* ldgmg_handle;

/* Problem statement (Section 2.1 / 3.1) and solver options (Section 2.2-2.4). */
typedef struct {
  int dim;            /* 2 or 3                                                   */
  int n;              /* elements per side; the grid is n^dim on (0,1)^dim        */
  int p;              /* polynomial degree, 1..5 (Q_p tensor-product space)       */
  int basis;          /* LDGMG_BASIS_*                                            */
  int system;         /* LDGMG_POISSON (scalar / interface) | LDGMG_STOKES        */
  int gamma;          /* Stokes form: 0 standard, 1 stress                        */
  int bc[6];          /* per box face (x-, x+, y-, y+, z-, z+): LDGMG_BC_*        */
  const double* mu;   /* host, n^dim per-element viscosities; NULL means all 1.
                         Read during setup only.                                  */
  double tau0;        /* velocity / scalar penalty: tau_F = tau0 mu_F / h         */
  double cp;          /* Stokes pressure penalty: c_p h / max(mu_L, mu_R)         */
  int smoother;       /* LDGMG_SMOOTH_*                                           */
  int sai_level;      /* l of SAI_l (pattern of A^l), 0..2                        */
  int order;          /* LDGMG_ORDER_*                                            */
  int nu1, nu2;       /* pre/post smoothing steps (paper: 3, 3)                   */
  double omega;       /* damping (Jacobi 0.8, coloured GS 1.0); <= 0 -> default   */
  double zeta;        /* Stokes balancing weight (tab:zeta); <= 0 -> tab:zeta     */
  int precision;      /* LDGMG_FP64 | LDGMG_FP32 | LDGMG_BF16S (block storage)   */
  int nthreads;       /* host threads for the setup; <= 0 -> hardware count      */
  size_t hbm_budget;  /* refuse ldgmg_upload above this many bytes; 0 = no limit */
  int storage;        /* LDGMG_STORE_* (default AUTO)                            */
  /* Unsteady Stokes (Section 3.4.4, eq:govern1unsteady, eq:blockformunsteady):
   * delta > 0 adds (1/delta) M_rho to every velocity block on every level
   * (M_rho: density-weighted block mass, coarsened as I^T M_rho I, delta the
   * same on every level; the paper takes delta = 0.1 h); delta = 0 (default):
   * steady.  The pressure penalty then uses mu + rho h^2 / delta in place of
   * mu, blending c_p h / mu (viscous limit) and c_p delta / (rho h)
   * (projection limit).  rho: host, n^dim per-element densities, NULL means
   * all 1; read during setup only.  Stokes only (EINVAL otherwise). */
  const double* rho;
  double delta;
  /* Where the setup solves the balanced SAI least-squares problems (Section
   * 2.3.3; its cache of identical problems, Section 4): 0 (default) on the
   * host; 1 on the current HIP device, in FP64, batched by shape (normal
   * equations with one refinement step, rocBLAS / rocSOLVER), the host taking
   * any problem the device declines (failed Cholesky, non-finite solution,
   * refinement step above 1e-8 of the solution).  With 1, ldgmg_setup_host
   * and ldgmg_rebuild_smoother need a GPU. */
  int setup_device;
  /* Device memory of the handle.  NULL (the default): hipMalloc / hipFree.
   * Otherwise every device buffer the handle owns (what ldgmg_upload
   * allocates, its temporary upload buffers, and the batch and GMRES
   * workspaces made by later calls) is taken with dev_alloc(bytes, alloc_ctx),
   * which returns device memory of the current device aligned to 256 bytes, or
   * NULL (the call then fails with LDGMG_ENOMEM); it is handed back with
   * dev_free(ptr, alloc_ctx) by ldgmg_unload / ldgmg_destroy, and temporary
   * upload buffers once the upload's stream has drained.  Both or neither
   * (else LDGMG_EINVAL).  The callbacks are called from the calling thread of
   * the entry point and must not call into the library.  For callers whose
   * allocator accounts for device memory (a caching allocator of a tensor
   * framework): hierarchies then count in its budget, and evicting one returns
   * its memory to that allocator without a device-wide synchronisation. */
  void* (*dev_alloc)(size_t bytes, void* alloc_ctx);
  void (*dev_free)(void* ptr, void* alloc_ctx);
  void* alloc_ctx;
} ldgmg_problem;

typedef struct {
  int iters;               /* Krylov iterations performed                          */
  int converged;           /* 1 if the stopping test was met                       */
  double rel_res_true;     /* ||b - A x||_2 / ||b||_2 in FP64 on the device        */
  double rel_res_krylov;   /* final Krylov-native stopping quantity                */
  double eta;              /* eq:eta from the Krylov-native residual history       */
  double* history;         /* host, caller-owned, may be NULL                      */
  int history_cap;         /* capacity of history                                   */
  int history_len;         /* entries written                                      */
  int vcycles;             /* V-cycle applications                                 */
} ldgmg_info;

/* Fill *p with the paper's defaults: Poisson, Legendre basis, Dirichlet on all
 * faces, tau0 = 1, cp = 0.1, SAI_1, OI, nu1 = nu2 = 3, FP32 V-cycle. */
int ldgmg_problem_default(ldgmg_problem* p);

/* Device bytes ldgmg_upload would allocate for this problem (no allocation, no
 * setup work beyond sizes).  Used for admission by HBM budget. */
int ldgmg_estimate_bytes(const ldgmg_problem* p, size_t* bytes);

/* Host setup (FP64): LDG assembly, factor coarsening (Section 2.2), smoother
 * construction (block inverses, colouring, balanced SAI with a cache of
 * identical least-squares problems), bottom pseudo-inverse.  Needs no GPU.
 * *out receives a new handle owning all host data. */
int ldgmg_setup_host(const ldgmg_problem* p, ldgmg_handle* out);

/* A new host hierarchy for problem p built from src: src's operators on every
 * level, transfers and bottom pseudo-inverse are copied and only the smoother
 * of p (smoother, sai_level, order, nu1, nu2, omega, zeta) is built; precision,
 * storage, nthreads and hbm_budget are taken from p.  p must describe the same
 * discrete problem as src (dim, n, p, basis, system, gamma, bc, tau0, cp and
 * equal viscosity values), else LDGMG_EINVAL.  Needs no GPU; src is unchanged.
 * For switching smoothers without repeating the assembly and the bottom
 * eigendecomposition. */
int ldgmg_rebuild_smoother(ldgmg_handle src, const ldgmg_problem* p, ldgmg_handle* out);

/* Copy a host-built hierarchy to the current HIP device (allocating with
 * hipMalloc) in the handle's precision; fails with LDGMG_ENOMEM above the
 * problem's hbm_budget. */
int ldgmg_upload(ldgmg_handle h, void* stream);

/* ldgmg_setup_host followed by ldgmg_upload. */
int ldgmg_setup(const ldgmg_problem* p, void* stream, ldgmg_handle* out);

/* Free the handle's device memory (levels, Krylov and batch workspaces); the
 * caller first synchronises the streams that used the handle, as before
 * ldgmg_destroy.  The host hierarchy stays, so a later
 * ldgmg_upload restores the handle without repeating the setup.  Until then
 * every call that needs device data returns LDGMG_ESTATE.  A handle that holds
 * no device data is left as it is. */
int ldgmg_unload(ldgmg_handle h);

/* CG guard for the solves of this handle (single and batched): when enabled,
 * CG stops at once, unconverged (LDGMG_ENOCONV), as soon as r^T V r <= 0 or
 * p^T A p <= 0, i.e. the V-cycle (or A) shows it is not positive definite on
 * the Krylov space; info holds the iterations done and the residual reached.
 * Off by default: plain preconditioned CG (Section 2.2), which can still
 * converge with such a preconditioner.  For callers that switch smoothers on
 * failure (serving).  Kept across ldgmg_unload / ldgmg_upload. */
int ldgmg_cg_guard(ldgmg_handle h, int enable);

/* CG solves of this handle (ldgmg_solve with LDGMG_CG) replayed from a HIP
 * graph: check_every = 0 (the default) launches every kernel of every
 * iteration from the host and synchronises once per iteration to test
 * convergence; check_every = k >= 1 captures one iteration of the recurrence
 * of Section 2.2 (the operator apply, the updates, the V-cycle of Algorithm 1
 * and the inner products) in a graph on the first such solve and replays it k
 * times between host synchronisations.  The convergence test runs on the
 * device: once the recurrence stops (||r|| <= rtol ||b||, maxit, the guard of
 * ldgmg_cg_guard, or a non-finite residual) the step length is 0, so the up to
 * k - 1 replays left leave x and r unchanged.  The results (iterations,
 * solution, residual history) equal those of the eager recurrence; the
 * replays after the stop cost device time only.  For right-hand sides whose
 * solves are bound by launch latency (small grids).  The graph uses the
 * handle's own vectors and is captured again after ldgmg_fp32_products,
 * ldgmg_cg_guard or ldgmg_upload; solves with ldgmg_profile on, maxit above
 * 4096 or GMRES stay eager.  Solves of one handle must not overlap (as for
 * every solve).  Batched and streamed solves are not affected. */
int ldgmg_cg_graph(ldgmg_handle h, int check_every);

/* FP32 products for the V-cycle of this handle: where a level is tiled
 * (ldgmg_level_storage), its operator and smoother applies (A, B, B^T, and the
 * block inverses of Jacobi) multiply on the FP32 matrix cores: the stored FP32
 * or BF16 entries exactly, the vector entries rounded to FP32 to nearest, sums
 * in FP32; the result is then combined with the FP64 vectors in FP64
 * (out = alpha y + beta z).  A precision choice of this library (the
 * method itself is stated in exact arithmetic): the V-cycle is only the
 * preconditioner, while the outer Krylov iteration, its operator, the
 * transfers and the bottom solve stay FP64.  The V-cycle is then no longer
 * one fixed linear operator (the rounding of its input varies), so CG can
 * need more iterations at high coefficient contrast.  With an SAI smoother,
 * on levels whose A and B are both tiled and whose block size is a multiple of
 * 16, the smoothing residual (consumed only by the B or B^T apply, which rounds
 * it to FP32 anyway) is written in FP32, and the smoother applies and the
 * prolongation keep an FP32 copy of the iterate beside it, which the operator
 * applies read (the same operand values as rounding the FP64 iterate): two
 * per-level buffers that ldgmg_upload allocates for such levels whether or not
 * this mode is on (N * 8 bytes, counted by ldgmg_upload_bytes).  Where a BF16
 * smoother matrix (BF16S precision, 32 | bs) reads that FP32 residual, its
 * products run on the BF16 matrix cores instead: each FP32 entry is split
 * into three BF16 parts (hi + mid + lo, by truncation; exact for entries of
 * magnitude at least 2^-103, below that the last part loses less than 2^-133),
 * so every product of a stored BF16 entry and a part is exact and the sums are
 * FP32, as on the FP32 matrix cores (a different summation order; the error
 * bound counts 3n summed terms in place of n).  Off by default; needs FP32 or BF16S
 * precision (LDGMG_EINVAL otherwise).  Kept across ldgmg_unload /
 * ldgmg_upload. */
int ldgmg_fp32_products(ldgmg_handle h, int enable);

/* Device bytes the handle holds now (0 when it holds no device data): what
 * ldgmg_upload allocated plus the batch workspace once a batched call made it. */
int ldgmg_device_bytes(ldgmg_handle h, size_t* bytes);

/* Device storage chosen for one level (needs device data): number of distinct
 * blocks stored for A and for the smoother matrix when pooled, 0 when that
 * matrix is expanded (every slot holds its block); *tiled: bit 0 A, bit 1 the
 * smoother matrix, set when tiled.  Any output may be NULL. */
int ldgmg_level_storage(ldgmg_handle h, int level, int* pool_A, int* pool_S, int* tiled);

/* Device bytes ldgmg_upload will allocate for this host hierarchy (exact for
 * its storage choices; the batch workspace of the batched calls not included). */
int ldgmg_upload_bytes(ldgmg_handle h, size_t* bytes);

/* Sizes: fine-level unknowns, unknowns per element, number of levels. */
int ldgmg_sizes(ldgmg_handle h, long long* ndofs, int* bs, int* nlevels);

/* Per-level sizes: elements per side, element count, stored blocks of A,
 * stored blocks of the smoother matrix (B for SAI, D^-1 otherwise), colours. */
int ldgmg_level_info(ldgmg_handle h, int level, int* n, int* nelem, int* nnzb_A,
                     int* nnzb_S, int* ncolours);

/* Volume load b_K[a] = int_K f psi_a (the f part of b_h, Section 2.1), from f
 * sampled at the nq^dim tensor Gauss-Legendre points of every element
 * (host array [n^dim][nq^dim], points with the x index fastest), written to
 * b_dev (device, FP64, fine-level layout).  Scalar problems only. */
int ldgmg_rhs_volume(ldgmg_handle h, const double* f_qp_host, int nq, double* b_dev,
                     void* stream);

/* x = V b: one V-cycle of Algorithm 1 with zero initial guess on the fine
 * level.  b_dev, x_dev: device FP64, fine-level layout (ndofs entries). */
int ldgmg_vcycle(ldgmg_handle h, const double* b_dev, double* x_dev, void* stream);

/* Solve A x = b from x0 = 0 with the V-cycle as preconditioner of CG
 * (krylov = LDGMG_CG; needs a symmetric V) or of left-preconditioned GMRES
 * (LDGMG_GMRES, no restart, at most min(maxit, 200) iterations).  Stops when
 * ||r||_2 <= rtol ||b||_2 (CG, FP64 recursive residual) or
 * ||V r||_2 <= rtol ||V b||_2 (GMRES).  Returns LDGMG_ENOCONV if maxit is hit
 * or, with ldgmg_cg_guard enabled, at a CG breakdown.  info may be NULL.
 *
 * Singular operators (Section 3.1: the Stokes pressure is defined up to a
 * constant; likewise a scalar problem without a Dirichlet face): the kernel of
 * constants found at upload (ldgmg_kernel) is handled by projecting b on the
 * range, b' = b - sum_i (b . k_i) k_i with orthonormal kernel vectors k_i,
 * solving A x = b', and returning the solution whose kernel components have
 * zero mean (for Stokes with velocity Dirichlet data: int p = 0).  The
 * residuals in info are relative to ||b'||.  With ldgmg_rhs_check set, a
 * right-hand side with |b . k_i| > tol ||b|| is refused with LDGMG_ESINGULAR
 * before any iteration. */
int ldgmg_solve(ldgmg_handle h, const double* b_dev, double* x_dev, int krylov,
                double rtol, int maxit, ldgmg_info* info, void* stream);

/* Consistency check of right-hand sides for singular operators: tol > 0
 * makes ldgmg_solve / ldgmg_solve_batch return LDGMG_ESINGULAR when
 * |b . k_i| > tol ||b||_2 for a unit kernel vector k_i (Section 3.1: A x = b
 * has a solution only for b orthogonal to the kernel of the symmetric A);
 * tol = 0 (the default) projects every b silently.  Kept across
 * ldgmg_unload / ldgmg_upload.  No effect on nonsingular operators. */
int ldgmg_rhs_check(ldgmg_handle h, double tol);

/* Kernel of the fine operator found at upload (needs device data): *count
 * unit vectors (0 for a nonsingular operator), each the constant function of
 * one component (the pressure of Stokes; the scalar field, or the velocity
 * components, when no box face is Dirichlet), kept only if
 * max |A k| <= 1e-10 max (|A| |k|) over the rows.  host_out: NULL, or *count * ndofs doubles,
 * receiving the vectors (fine-level layout). */
int ldgmg_kernel(ldgmg_handle h, int* count, double* host_out);

/* Batched serving step: k right-hand sides, right-hand side q on hierarchy
 * hs[q] (the same handle may appear several times; handles may differ in
 * size and problem).  Every right-hand side is solved as by ldgmg_solve with
 * `krylov` (same stopping rule, kernel handling and info).  Right-hand sides
 * of one handle share the work: with LDGMG_CG they run in groups of up to 16,
 * each with its own preconditioned CG recurrence (a right-hand side that
 * converges is frozen) while every V-cycle stage and operator apply streams
 * each matrix block once for the group; with LDGMG_GMRES they run one after
 * the other.  b_dev / x_dev: host arrays of k device FP64 pointers
 * (fine-level layout of their handle).  infos: k entries or NULL; vcycles
 * counts the V-cycles applied to that right-hand side.  Returns LDGMG_ENOCONV
 * if any right-hand side is not converged.  Handles must be distinct or
 * identical, never two handles sharing device data, and all on the current
 * device.  A handle's first batched CG call allocates 5 fine-level vector
 * sets plus 4 on every level, each of 8 vectors (16 once more than 8
 * right-hand sides share a group). */
int ldgmg_solve_batch(const ldgmg_handle* hs, const double* const* b_dev, double* const* x_dev, int k,
                      int krylov, double rtol, int maxit, ldgmg_info* infos, void* stream);

/* Continuous batching on one hierarchy (serving): CG solves whose right-hand
 * sides are handed over while others are in flight.  Up to `slots` (1..16)
 * preconditioned CG recurrences run at once, each exactly that of
 * ldgmg_solve with LDGMG_CG on its own right-hand side (same stopping rule,
 * guard and kernel handling), while every V-cycle stage and operator apply
 * streams each matrix block once for all slots in use.  Before every V-cycle
 * stage the library fills free slots by calling
 *     next(ctx, &b_dev, &x_dev, &tag)
 * which returns 1 with a right-hand side, its solution vector (device FP64,
 * fine-level layout, valid until done() reports that tag) and a caller tag,
 * or 0 when nothing is waiting now (it is asked again at the next stage while
 * a slot is free, so right-hand sides that arrive meanwhile are admitted).  A
 * new right-hand side joins the batch at that stage with its first V-cycle.  When a recurrence stops (converged, maxit, guarded
 * breakdown) its solution is written to x_dev, then
 *     done(ctx, tag, status, &info)
 * is called (status LDGMG_OK or LDGMG_ENOCONV; info as ldgmg_solve fills
 * it) and the slot is free again.  Returns when no slot is in flight and
 * next() returns 0: LDGMG_ENOCONV if any right-hand side did not converge.  The callbacks run on the calling thread, between the library's
 * launches on `stream`, and must not call into the library with this
 * handle.  Workspace as for ldgmg_solve_batch with `slots` right-hand sides. */
int ldgmg_solve_stream(ldgmg_handle h, int slots, double rtol, int maxit,
                       int (*next)(void* ctx, const double** b_dev, double** x_dev, long long* tag),
                       void (*done)(void* ctx, long long tag, int status, const ldgmg_info* info),
                       void* ctx, void* stream);

/* x_q = V b_q for k <= 16 right-hand sides with one batched V-cycle. */
int ldgmg_vcycle_batch(ldgmg_handle h, const double* const* b_dev, double* const* x_dev, int k,
                       void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * batched V-cycle as ldgmg_vcycle_batch (same kernels, same results), with
 * its per-level batch vectors taken from a static device array of 128 MiB
 * that the library holds on each GPU until the process ends, instead of the
 * handle's batch workspace (which ldgmg_vcycle_batch allocates on its first
 * call).  Allocates nothing: no hipMalloc / hipFree, no allocator callback.
 * Needs 4 k sum_l N_l doubles (N_l the unknowns of level l), at most 16M;
 * larger requests fail with LDGMG_EINVAL.  Every call on one GPU shares that
 * array: calls that overlap on one GPU (other streams, other handles, other
 * threads) race and must be serialised by the caller.  Nothing in the array
 * needs to start at zero (every vector is written before it is read). */
int ldgmg_vcycle_batch_noalloc(ldgmg_handle h, const double* const* b_dev, double* const* x_dev, int k,
                               void* stream);

/* Single operations of the V-cycle on one level, for checking each kernel.
 * in1/in2/out are device FP64 vectors of the level (ne*bs entries; the
 * coarse vector of RESTRICT / PROLONG_ADD has the next level's size).
 *   LDGMG_OP_RESIDUAL    out = in2 - A in1                  (b - A x)
 *   LDGMG_OP_APPLY_A     out = A in1
 *   LDGMG_OP_APPLY_S     out = S in1, S = B (SAI) or D^-1 (Jacobi / GS)
 *   LDGMG_OP_APPLY_ST    out = S^T in1
 *   LDGMG_OP_SMOOTH_FWD  out = in1 after one forward smoothing step with b = in2
 *   LDGMG_OP_SMOOTH_REV  out = in1 after one reverse smoothing step with b = in2
 *   LDGMG_OP_RESTRICT    out (level+1) = I^T in1 (level)
 *   LDGMG_OP_PROLONG_ADD out (level) += I in1 (level+1)
 *   LDGMG_OP_BOTTOM      out = A^+ in1 on the bottom level
 *   LDGMG_OP_APPLY_A64   out = A in1 in FP64 on the fine level (Krylov operator)
 * in2 is read only by RESIDUAL and the SMOOTH ops. */
enum { LDGMG_OP_RESIDUAL = 0, LDGMG_OP_APPLY_A = 1, LDGMG_OP_APPLY_S = 2,
       LDGMG_OP_APPLY_ST = 3, LDGMG_OP_SMOOTH_FWD = 4, LDGMG_OP_SMOOTH_REV = 5,
       LDGMG_OP_RESTRICT = 6, LDGMG_OP_PROLONG_ADD = 7, LDGMG_OP_BOTTOM = 8,
       LDGMG_OP_APPLY_A64 = 9 };
int ldgmg_level_op(ldgmg_handle h, int level, int op, const void* in1, const void* in2,
                   void* out, void* stream);

/* Export host-side setup data (FP64) for checking.  what:
 *   LDGMG_EXPORT_A     block-sparse A of the level
 *   LDGMG_EXPORT_S     smoother matrix (B for SAI, block-diagonal D^-1 otherwise)
 *   LDGMG_EXPORT_PINV  bottom pseudo-inverse (dense, row-major; level ignored)
 * Block-sparse exports fill row_ptr [nelem+1], col [nnzb] and blocks
 * [nnzb][bs][bs] (row-major inside a block).  Call with blocks == NULL to get
 * *nnzb (and *dense_n for PINV) only.  Host pointers, caller-owned. */
enum { LDGMG_EXPORT_A = 0, LDGMG_EXPORT_S = 1, LDGMG_EXPORT_PINV = 2 };
int ldgmg_export(ldgmg_handle h, int level, int what, int* row_ptr, int* col,
                 double* blocks, int* nnzb, int* dense_n);

/* Colours of the multi-coloured Gauss-Seidel smoother (host int[nelem]). */
int ldgmg_export_colours(ldgmg_handle h, int level, int* colours);

/* Setup statistics: unique SAI least-squares problems solved on the level and
 * the level's setup time in seconds (with setup_device = 1, the problems that
 * the device solved are reported by ldgmg_setup_stats_device). */
int ldgmg_setup_stats(ldgmg_handle h, int level, int* sai_unique, double* seconds);

/* Unique SAI least-squares problems of the level solved on the device
 * (setup_device = 1) and by Householder QR on the host (declined by the
 * normal equations), and the seconds the level's SAI least-squares solves
 * took (device and host together). */
int ldgmg_setup_stats_device(ldgmg_handle h, int level, int* sai_device, int* sai_qr, double* sai_seconds);

/* Kernel timing of the fine level (diagnostics, for roofline measurements).
 * While enabled, every block-sparse launch on level 0 is bracketed by HIP
 * events on the stream it is launched on.  kind: 0 = A (residual / apply),
 * 1 = smoother matrix forward, 2 = smoother matrix transposed, 3 = FP64 Krylov
 * operator, 4 = fused block-inverse smoothing (A and D^-1).
 * ldgmg_profile_read synchronises the recorded events and returns the launch
 * count and the summed duration in milliseconds of one kind; enabling again
 * clears the records.  At most 4096 launches are recorded per enable. */
int ldgmg_profile(ldgmg_handle h, int enable);
int ldgmg_profile_read(ldgmg_handle h, int kind, int* count, double* total_ms);

/* Release all host and device memory of the handle. */
int ldgmg_destroy(ldgmg_handle h);

const char* ldgmg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LDGMG_H */
