/* hpdg.h -- C ABI of the MI355X hp-DG subspace-correction solver.
 *
 * Problem (Sec. 2, eq. fe-problem): find u_h in V_h with A(u_h, v) = (f, v)
 * for all v in V_h, V_h the discontinuous space of tensor polynomials of
 * degree p_K on each leaf K of an irregular quadtree (2D) / octree (3D) mesh
 * of [0,1]^d, A the SIPG form (Sec. 2) or the BR2 form (Sec. 4.4) of
 * -div(k grad u) = f with homogeneous Dirichlet data. The system is solved
 * by CG (Sec. 4.1) preconditioned with B = B_J + B_E + P T_C P^T (Sec. 3.1,
 * eq. TB, Sec. 3.4): point Jacobi on V_J, exact block solves on the V_e,
 * and one AMG V-cycle on the low-order-refined conforming matrix.
 *
 * Conventions (all entry points):
 *  - Return value: HPDG_OK (0) or a negative hpdg_status; hpdg_last_error()
 *    gives a message for the calling thread. Argument errors are detected
 *    before any device work is queued.
 *  - Vectors passed to the operator calls are DEVICE pointers owned by the
 *    caller; the library never frees them. DOFs are element-major in input
 *    leaf order; inside an element the Gauss-Lobatto nodes are ordered
 *    lexicographically with x fastest. With nrhs > 1 vectors are
 *    RHS-interleaved: v[dof * nrhs + r].
 *  - stream: a hipStream_t passed as void*; NULL means the null stream.
 *    Calls are stream-ordered. A handle is not thread-safe.
 *  - Mesh input arrays are HOST pointers, copied during the call.
 */
#ifndef HPDG_H
#define HPDG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HPDG_OK = 0,
  HPDG_E_INVALID = -1,       /* bad argument or mesh */
  HPDG_E_NOMEM = -2,         /* host or device allocation failed */
  HPDG_E_HIP = -3,           /* HIP runtime error */
  HPDG_E_NOT_SPD = -4,       /* CG breakdown: p'Ap <= 0 or r'z <= 0 */
  HPDG_E_NOT_CONVERGED = -5, /* maxit reached */
  HPDG_E_UNSUPPORTED = -6,
  HPDG_E_BUSY = -7           /* batch admission: no free slot (retry later) */
} hpdg_status;

typedef struct hpdg_mesh hpdg_mesh;
typedef struct hpdg_operator hpdg_operator;
typedef struct hpdg_batch hpdg_batch;

const char* hpdg_last_error(void);

/* Mesh of leaves (Sec. 2: elements K with affine maps T_K and degree p_K;
 * Sec. 4.3: piecewise-constant coefficient).
 *  dim     2 or 3
 *  n_base  the base grid has n_base^dim cells on [0,1]^dim
 *  level   [n_elem] refinement level >= 0
 *  anchor  [n_elem*dim] lower corner in units of 1/(n_base*2^level)
 *  degree  [n_elem] polynomial degree, 1..8
 *  kcoef   [n_elem] coefficient k > 0
 * Validation: the leaves must tile [0,1]^dim exactly (no overlap, no gap).
 * On success *out owns a host-side topology (faces, neighbours). */
hpdg_status hpdg_setup_mesh(int dim, int n_base, int64_t n_elem, const int32_t* level,
                            const int32_t* anchor, const int32_t* degree, const double* kcoef,
                            hpdg_mesh** out);
/* ndof: number of DG unknowns; nface: faces of the skeleton (Sec. 2,
 * sub-faces counted separately, boundary faces included); max_level_jump:
 * largest level difference across a face. Any output pointer may be NULL. */
hpdg_status hpdg_mesh_info(const hpdg_mesh* mesh, int64_t* ndof, int64_t* nface, int* max_level_jump);
void hpdg_mesh_destroy(hpdg_mesh* mesh);

typedef struct {
  int form;          /* 0 SIPG (Sec. 2), 1 BR2 (Sec. 4.4) */
  int penalty_rule;  /* SIPG sigma = eta*k_e*pi(p_e)/h_e: 0 -> pi = (p+1)^2, 1 -> pi = p^2 (Sec. 2) */
  double eta;        /* SIPG eta; BR2 eta (<= 0: 1 + largest face count of an element) */
  int prec_fp32;     /* 0: FP64 preconditioner; 1: FP32 preconditioner, FP64 CG */
  int remark_relax;  /* 1: add the Remark-cases DOFs to V_J (Sec. 3.3); default 0 */
  int jb_only;       /* 1: simplified J_B + B_C (Sec. 4.1): point Jacobi on all of V_B */
  int max_block;     /* > 0: a V_e larger than this is handled by point Jacobi */
  int max_nrhs;      /* >= 1 and a divisor of 256: largest nrhs accepted by the operator calls */
  int host_only;     /* 1: build only the host-side setup data (readable with hpdg_export) and
                        touch no GPU; the operator calls then fail with HPDG_E_UNSUPPORTED */
  int no_prec;       /* 1: the DG operator only (no preconditioner setup); hpdg_apply_B and
                        hpdg_pcg_solve then fail with HPDG_E_UNSUPPORTED */
  int graph;         /* 1: PCG iterations are captured once per (chunk length, nrhs, x) into
                        HIP graphs and replayed (same kernels, same results) */
  int setup_threads; /* host threads for the setup's sparse products (0: all hardware
                        threads, 1: serial); results do not depend on it */
  int auto_cycle;    /* 1: at upload, without timing, every AMG level with at most 256K
                        nonzeros in the fused form and the dense tail on the level above
                        the coarsest when it has at most 512 rows (see hpdg_operator_tune):
                        fewer launches per V-cycle, for callers that do not run the
                        autotuner (many small solves); the same operator, other rounding */
} hpdg_operator_opts;

/* Builds the operator and the preconditioner (host setup, then upload):
 * faces and penalties, diag(A) and the V_J / V_e split (Sec. 3.3), the V_e
 * blocks and their inverses, the conforming prolongation P (Sec. 3.4), the
 * LOR matrix A~_C = P^T A~ P and its AMG hierarchy. The mesh may be destroyed
 * afterwards. The operator owns all its device memory until destroy. Uploads
 * are synchronous; the call ends with a synchronisation of `stream` only, so
 * setups of different operators may run in parallel host threads while other
 * operators solve on their own streams. */
hpdg_status hpdg_setup_operator(const hpdg_mesh* mesh, const hpdg_operator_opts* opts, void* stream,
                                hpdg_operator** out);
void hpdg_operator_destroy(hpdg_operator* op);

/* b = M f: load vector (f, v) of Sec. 2 for f given by its values at the DG
 * nodes (exact element mass matrices). f_nodal, b: device, ndof*nrhs. */
hpdg_status hpdg_rhs(hpdg_operator* op, const double* f_nodal, double* b, int nrhs, void* stream);

/* y = A x: matrix-free DG operator (Sec. 4.1, component 1): sum-factorised
 * volume terms and the SIPG/BR2 face terms, FP64. x, y: device, ndof*nrhs,
 * must not alias. */
hpdg_status hpdg_apply_A(hpdg_operator* op, const double* x, double* y, int nrhs, void* stream);

/* z = B r (Sec. 3.1 with eq. TB; Sec. 4.1 components 2-5), in the operator's
 * preconditioner precision, inputs and outputs FP64. r, z: device,
 * ndof*nrhs, must not alias. */
hpdg_status hpdg_apply_B(hpdg_operator* op, const double* r, double* z, int nrhs, void* stream);

/* z = B r like hpdg_apply_B, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the call allocates nothing. B's work vectors (the
 * preconditioner-precision copies of r and z and the V-cycle vectors of every
 * AMG level) are carved out of a static 64 MiB device array, one per GPU, that
 * the library holds until the process ends; the operator's own matrices are
 * only read. Same kernels, same results as hpdg_apply_B.
 *  - Limit: the work vectors take (ndof [+ ndof in FP32 mode] + 4 x the rows of
 *    every AMG level) x nrhs values of the preconditioner's precision, each
 *    vector rounded up to 256 bytes; more than 64 MiB returns HPDG_E_INVALID
 *    before any device work (use hpdg_apply_B then).
 *  - The array is shared by every call on a GPU and keeps the last call's
 *    contents; no part of it needs to start at zero (each call writes every
 *    word it reads first). Calls that overlap in time on one GPU (other
 *    streams or host threads) race on it: the caller orders them.
 *  - Runs on the current device (the one the operator was set up on); the
 *    first call on a device looks up the array's address there.
 *  - Unlike hpdg_apply_B it may run while the operator has a solve in flight,
 *    since it does not touch the operator's work vectors.
 * r, z: device, ndof*nrhs, must not alias. */
hpdg_status hpdg_apply_B_noalloc(hpdg_operator* op, const double* r, double* z, int nrhs, void* stream);

typedef struct {
  int iters, converged;
  double rel_res;       /* recurrence residual ||r_k|| / ||b|| */
  double true_rel_res;  /* ||b - A x|| / ||b|| recomputed in FP64 at the end */
  double lambda_min, lambda_max, cond_est;  /* Lanczos from the CG coefficients */
  double t_solve_s;     /* host wall time of the solve */
  double t_setup_s;     /* host wall time of the operator's setup (hpdg_setup_operator, plus
                           hpdg_operator_upload for a host_only operator) */
} hpdg_solve_info;

/* PCG (Sec. 4.1) on T = BA, stopping at ||r_k||_2 <= rtol ||b||_2 (per RHS).
 * x holds the initial guess on entry and the result on exit (device,
 * ndof*nrhs). Blocks the host until done. info: host array [nrhs] or NULL.
 * The flags are read back after the first iteration and then every 4; the
 * Lanczos estimate uses the first 2048 iterations.
 * Returns HPDG_E_NOT_SPD on a breakdown and HPDG_E_NOT_CONVERGED at maxit
 * (x then holds the last iterate and info is filled). */
hpdg_status hpdg_pcg_solve(hpdg_operator* op, const double* b, double* x, int nrhs, double rtol, int maxit,
                           void* stream, hpdg_solve_info* info);

/* Device memory of an operator. An operator set up with host_only holds only
 * host data; hpdg_operator_upload copies it to the device (synchronous
 * copies, then a synchronisation of `stream`) and makes it usable for every
 * call. Idempotent. Different operators may be uploaded from different host
 * threads at once. */
hpdg_status hpdg_operator_upload(hpdg_operator* op, void* stream);

/* Exact device bytes the operator holds once uploaded (computed by a
 * counting pass over the upload when it is not on the device yet); the
 * figure a server admits requests by. */
hpdg_status hpdg_operator_device_bytes(hpdg_operator* op, int64_t* bytes);

/* Autotuner for the one-RHS path: for P^T and every AMG level matrix A_l,
 * R_l, P_l, times y = A x under each row binning (rows longer than 64, 128,
 * 256 or 512 entries or no threshold get a wavefront each; the others 1, 2,
 * 4, 8 or 16 lanes, each lane taking 4-entry chunks) on `stream` and keeps
 * the fastest. Changes the summation order and
 * so the last bits of B r; drops captured graphs. With no_prec only the
 * element kernel is tuned (in 2D its tiles and, for max_nrhs > 1, its
 * right-hand-side form: kinds 4 and 6). In 2D it also picks, for the element kernel, the
 * elements per workgroup (1 or 2) and the face records staged per pass (8,
 * 16 or 32); the results do not depend on them. report: cap rows of 8 int64
 * (kind 0 A / 1 R / 2 P / 3 P^T / 4 element kernel / 5 fused V-cycle level /
 * 6 right-hand sides per element-kernel item, at the largest nrhs (chosen
 * lanes 0: a lane per right-hand side, one wavefront per element and 64
 * RHS, for the degrees up to the threshold column's, the others grouped;
 * 9 there: every degree on the lane form in two launches; 10: every degree
 * in one launch, elements by decreasing cost within each XCD's share; the
 * threshold column holds nrhs otherwise) /
 * 7 lanes per V_e block row for the one-RHS block solves (the threshold
 * column holds 1 when they run as a workgroup per block with the block's r
 * staged in LDS, 0 when their rows run inside the B front) / 8 dense tail of the
 * V-cycle on the level above the coarsest (chosen lanes 1 if kept) / 10 3D
 * element kernel dispatched by decreasing element cost (chosen lanes 1 if
 * kept; the threshold column holds the ns of that order) / 11 V_e block
 * solves on the operator's second stream, concurrent with the V-cycle
 * (chosen lanes 1 if kept; the threshold column holds the V-cycle level
 * after whose down-leg they start; rows and nnz hold ndof and the block
 * count),
 * level, rows (ndof), nnz (elements), chosen threshold (records per pass),
 * chosen lanes (elements per workgroup; 1 if the level is fused), ns before,
 * ns after); *n rows written. A fused level (one RHS, at most 4M nonzeros)
 * runs the V(1,1) steps of that level in two launches with the precomputed
 * products R (I - A D) and A P instead of four; it is kept only where it
 * measures faster, and its matrices add device memory. Its row holds the
 * lanes per row of the fused up-leg in the threshold column. */
hpdg_status hpdg_operator_tune(hpdg_operator* op, void* stream, int64_t* report, int cap, int* n);

/* Batch executor for serving (continuous batching on one GPU): up to
 * max_active (1..64) PCG solves, each on a stream of its own (default
 * priority, non-blocking), advance together in chunks of iterations. Every
 * reduction has a fixed order, so a solve gives bitwise the same result
 * alone or among others. A batch is driven from one host thread.
 *
 * admit: start the PCG of hpdg_pcg_solve (one RHS) for an uploaded operator
 *   with caller-owned device vectors b, x (x: initial guess) that stay
 *   untouched by the caller until the solve is retired. b must be complete
 *   (the caller synchronises the stream that wrote it). Returns HPDG_E_BUSY
 *   when every slot is taken; admission by device memory is the caller's
 *   policy, using hpdg_operator_device_bytes.
 * step: advance every solve whose last chunk has completed (enqueue the next
 *   chunk, the final FP64 residual, or retire it). Waits up to wait_us
 *   microseconds for progress; never blocks on the device otherwise.
 * poll: pop up to cap retired solves: tag, status (as hpdg_pcg_solve) and
 *   info. A retired operator may be reused or destroyed. Until then the
 *   operator, b and x must stay alive: destroying an admitted operator or
 *   freeing its vectors is invalid, and hpdg_pcg_solve and hpdg_apply_B on it
 *   return HPDG_E_INVALID (they would overwrite the work vectors of the
 *   solve in flight).
 * destroy: synchronises the batch's streams; solves still active are left
 *   unfinished and their operators may only be destroyed afterwards. */
hpdg_status hpdg_batch_create(int max_active, hpdg_batch** out);
void hpdg_batch_destroy(hpdg_batch* bt);
hpdg_status hpdg_batch_admit(hpdg_batch* bt, hpdg_operator* op, const double* b, double* x, double rtol, int maxit,
                             int64_t tag);
hpdg_status hpdg_batch_step(hpdg_batch* bt, int wait_us, int* n_active, int* n_done);
hpdg_status hpdg_batch_poll(hpdg_batch* bt, int cap, int64_t* tags, int* status, hpdg_solve_info* info, int* n);

/* Host copies of setup data, for tests. what:
 *  0 diag(A) [ndof] double      1 labels [ndof] int8 (0 interior, 1 V_J, 2 N)
 *  2 P as CSR: int64 nrows, ncols, nnz, then ptr[nrows+1] int64,
 *    idx[nnz] int32, val[nnz] double
 *  3 A~_C as CSR (same layout)  4 V_e blocks: int64 nblocks, ptr[nb+1] int64,
 *    dofs int64                 5 DG node coordinates [ndof*dim] double
 *  6 AMG level sizes: int64 nlevels, rows[nlevels], nnz of A[nlevels], nnz of
 *    the prolongation from the next coarser level[nlevels] (0 on the coarsest)
 *  7 summary: int64[10] = ndof, nconf, nblocks, max block, block entries,
 *    amg levels, nnz(A~_C), nnz(P), bytes of the face-matrix table, device
 *    bytes held by the operator
 *  8 inverses of the V_e blocks in FP64, row-major, concatenated in the
 *    order of item 4
 *  9 CG coefficients of the operator's last finished hpdg_pcg_solve, double:
 *    rows, stride (= max_nrhs), alpha[rows*stride], beta[rows*stride]
 *    (iteration-major, RHS c at offset c; beta of the last row unused);
 *    HPDG_E_INVALID before any finished solve
 *  100+l  AMG level-l matrix A_l as CSR;  200+l  AMG prolongator P_l as CSR;
 *  300+l  aggregate index of every row of level l, int64
 * bytes: in: capacity of buf; out: bytes needed. buf NULL queries the size. */
hpdg_status hpdg_export(const hpdg_operator* op, int what, void* buf, size_t* bytes);

#ifdef __cplusplus
}
#endif
#endif /* HPDG_H */
