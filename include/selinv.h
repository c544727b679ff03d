/*
 * selinv.h -- C ABI of the MI355X selected-inversion library.
 *
 * Method: Jacquelin, Lin, Jia, Zhao, Yang, "A Left-Looking Selected Inversion
 * Algorithm and Task Parallelism on Shared Memory Systems" (arXiv:1604.02528).
 * Given a sparse symmetric (real), complex-symmetric or Hermitian matrix A
 * and a symmetric fill-reducing permutation P, the library computes every
 * entry of B^{-1}, B = P A P^T, on the sparsity pattern of the L factor of B
 * (Alg. 1 / Alg. 2 outputs: the selected blocks A^{-1}_{I,J} with L_{I,J}
 * nonempty; the LDL^T specialization of Section 2.3 makes the upper triangle
 * the transpose of the lower one, and its Hermitian variant the conjugate
 * transpose).  For a real unsymmetric A with a symmetric pattern
 * (SELINV_LU64) it computes both triangles from the LU form of Alg. 1
 * (Section 2.1, with B = L D U unpivoted).
 *
 * Conventions shared by every entry point
 *  - Matrices: lower triangle incl. diagonal, CSC, 0-based, int64 indices,
 *    rows strictly increasing inside a column, diagonal present
 *    (structurally symmetric pattern, Section 2.1).
 *  - perm: new -> old (B[i,j] = A[perm[i], perm[j]]); NULL = identity.
 *    The paper permutes symmetrically without looking at values (Section 4).
 *  - Values: `batch` matrices with one pattern (the shifts H - z_l S of a
 *    pole expansion), laid out [batch][nnz] in rowind order.  Complex values
 *    (SELINV_C128, SELINV_H128) are interleaved (re, im) doubles.  For
 *    SELINV_C128 transposes are plain transposes (complex-symmetric,
 *    A = A^T); for SELINV_H128 (Hermitian, A = A^H, real diagonal) every
 *    transpose is a conjugate transpose: B = L D L^H, and a stored lower
 *    value that the permutation moves into B's upper triangle enters B's
 *    lower triangle conjugated.  SELINV_LU64 values are [batch][2 nnz]
 *    doubles: per matrix the nnz lower values A(rowind[e], j) in rowind
 *    order, then their mirrors A(j, rowind[e]) in the same order (the
 *    diagonal is taken from the first half).
 *  - Panels: supernode K (columns first(K)..last(K), width s, row set C(K) of
 *    size c, Eq. (newset)) owns a dense column-major (s + c) x s block whose
 *    rows are K's own columns followed by C(K).  Panels are concatenated in K
 *    order; one matrix of the batch occupies `panel_elems` scalars and matrix
 *    l starts at l * panel_elems.  The same layout is used for the factor
 *    panels and for the selected inverse X.  An SELINV_LU64 matrix holds two
 *    panel sets of that layout, one after the other (panel_elems counts
 *    both): the first holds L (unit, with D in the diagonal slots) and X =
 *    B^{-1} on the pattern of L, the second U^T and X^T on the same
 *    pattern.
 *  - Device memory is always allocated by the caller (sizes from
 *    selinv_sizes) and never freed by the library.  Device pointers are plain
 *    `void*` from hipMalloc (or a framework allocator on the same device).
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *  - Every function returns selinv_status; no C++ exception crosses the ABI.
 *    On error, selinv_last_error(ctx) explains it and selinv_error_info(ctx, k)
 *    gives integers (k = 0: column, k = 1: batch index) where meaningful.
 *    After an error, output buffers are undefined.  A context is not
 *    thread-safe; distinct contexts are independent.
 */
#ifndef SELINV_H
#define SELINV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct selinv_ctx selinv_ctx;

typedef enum {
  SELINV_R64 = 0,  /* real float64 */
  SELINV_C128 = 1, /* complex128, complex-symmetric */
  SELINV_H128 = 2, /* complex128, Hermitian (Section 2.3: conjugate transposes); no adjoint */
  SELINV_LU64 = 3  /* float64, unsymmetric values on a symmetric pattern (Alg. 1 in its LU form,
                      Section 2.1); level schedule only (gathered or dense X_{C,C}; no split
                      contractions or tune table), host factorization only; no adjoint, no Dt
                      output, no selinv_scatter */
} selinv_dtype;

typedef enum {
  SELINV_OK = 0,
  SELINV_EINVAL = 1,       /* bad argument (null pointer, size, option) */
  SELINV_EPATTERN = 2,     /* malformed CSC pattern or permutation */
  SELINV_ESINGULAR = 3,    /* zero or non-finite pivot (no pivoting is done) */
  SELINV_ENOMEM = 4,       /* host allocation failed or size overflow */
  SELINV_EDEVICE = 5,      /* HIP runtime error or device watchdog */
  SELINV_ESTATE = 6,       /* calls out of order (e.g. run before factor) */
  SELINV_EUNSUPPORTED = 7  /* dtype / mode not supported */
} selinv_status;

/* Scheduling of the selected-inversion traversal (root to leaves). */
typedef enum {
  SELINV_SCHED_PERSISTENT = 0, /* one launch; workgroups draw tickets of a topological order and wait on
                                  per-node dependency counters */
  SELINV_SCHED_LEVELS = 1,     /* one launch per etree depth and phase (the default: measured faster) */
  SELINV_SCHED_PUSH = 2        /* the paper's left-looking form (Alg. 2): per etree depth, root first,
                                  the depth's diagonal blocks (D), then every descendant's X_{C,I}
                                  updated with the depth's blocks (the O, I and ID updates of
                                  Eqs. (outerprod) and (innerprod)); measured against the pull form */
} selinv_sched;

typedef struct {
  int32_t max_super;   /* supernode size cap (Section 2.1: the definition may cap it); default 256 */
  int32_t dtype;       /* selinv_dtype */
  int32_t batch;       /* number of matrices sharing the pattern, >= 1 */
  int32_t sched;       /* selinv_sched */
  double relax;        /* explicit-zero budget of supernode chain amalgamation, 0 = maximal supernodes */
  int32_t nthreads;    /* host threads for the factorization; 0 = hardware concurrency */
  int32_t dense_min_c; /* nodes with |C(K)| >= this get a dense X_{C,C} buffer in the work area
                          (gathered once, then read by plain GEMM tiles); 0 = 256, < 0 = never */
  int64_t watchdog_ms; /* persistent schedule: budget of each single dependency wait, in ms (0 = 10000);
                          < 0: -watchdog_ms device clock ticks (a way to exercise the expiry path).  An
                          expired wait raises the device error flag, every workgroup exits, and
                          selinv_sync returns SELINV_EDEVICE; X is then undefined */
  int64_t dense_max_bytes; /* cap on those buffers for the whole batch; the threshold is doubled
                              until they fit (0 = 32 GiB).  Under SELINV_SCHED_LEVELS the buffers
                              of different etree depths share memory, so the cap applies to the
                              largest depth; under SELINV_SCHED_PERSISTENT to their sum */
  int32_t split_min_k; /* shortest contraction part when a node with too few GEMM-1 tiles to fill
                          the GPU splits its contraction over C(K) (0 = 320, < 0 = never split);
                          a quarter of it at etree depths whose tiles fill at most a quarter of
                          the GPU */
  int32_t adjoint;     /* 0 (default): the work area includes the adjoint's scratch (three panel-layout
                          arrays and three s x s arrays per matrix), so that selinv_backward can run;
                          < 0: left out (a smaller work area; selinv_backward returns EUNSUPPORTED) */
  const char *tune_cache; /* path of a tune table written by the autotuner (JSON, format
                             "selinv-tune-1"), or NULL.  Entries of this GPU target, ROCm version
                             and dtype choose, per bucket of supernode width s and |C(K)|, whether
                             X_{C,C} is gathered into a dense buffer, whether a dense node's GEMM-1
                             runs in the dense-loader kernel (level schedule), and split_min_k; they
                             override dense_min_c / split_min_k for the nodes they cover.  Read by
                             selinv_analyze (EINVAL on a malformed file); the string is copied */
} selinv_opts;

/* Fill `o` with defaults (cap 256, R64, batch 1, level schedule, relax 0.05).  relax = 0 gives the
   paper's maximal supernodes exactly; the default 0.05 is the fastest measured setting. */
void selinv_default_opts(selinv_opts *o);

/*
 * selinv_analyze -- symbolic analysis (Section 2.1, Eq. (newset)).
 *   n, colptr[n+1], rowind[colptr[n]]: A's lower pattern (host, borrowed).
 *   perm[n]: new -> old permutation or NULL.
 *   opts: NULL = defaults.
 * Computes B's pattern, the column elimination tree, column counts, the
 * supernode partition (maximal supernodes capped at max_super, optionally
 * relaxed along etree chains), C(K), the supernodal etree and the ancestor
 * index maps.  Errors: SELINV_EPATTERN (error_info(0) = offending column),
 * SELINV_EINVAL, SELINV_ENOMEM.  *out is owned by the caller and released
 * with selinv_destroy.
 */
selinv_status selinv_analyze(int64_t n, const int64_t *colptr, const int64_t *rowind,
                             const int64_t *perm, const selinv_opts *opts, selinv_ctx **out);

/* Host views of the symbolic data; pointers stay valid until selinv_destroy. */
typedef struct {
  int64_t n, nsuper, nnzL, panel_elems, batch, dtype;
  const int64_t *perm;       /* [n] new -> old */
  const int64_t *parent;     /* [n] column etree, -1 = root */
  const int64_t *colcount;   /* [n] nnz of each column of L, diagonal included */
  const int64_t *xsuper;     /* [nsuper+1] */
  const int64_t *sparent;    /* [nsuper] supernodal etree, -1 = root */
  const int64_t *rowptr;     /* [nsuper+1] C(K) = rowind_L[rowptr[K] .. rowptr[K+1]) */
  const int64_t *rowind_L;   /* sorted row sets */
  const int64_t *panel_off;  /* [nsuper] element offset of K's panel inside one matrix */
  /* canonical ancestor maps: segments of K are seg_ptr[K] .. seg_ptr[K+1]-1;
     segment g: owner seg_super[g], first index seg_start[g] into C(K); the
     panel-row positions inside the owner of rows C(K)[seg_start[g]:] are
     posarr[seg_posoff[g] ...] */
  const int64_t *seg_ptr, *seg_super, *seg_start, *seg_posoff;
  const int32_t *posarr;
  int64_t nseg, nposarr;
  double flops_exact;        /* sum_K 2c^2 s + 2 c s^2 over the maximal (relax = 0) partition, x4 for complex */
  double flops;              /* the same over the partition in use */
  int64_t depth;             /* supernodal etree height */
  int64_t tuned_nodes;       /* supernodes a tune-table entry applied to */
} selinv_symbolic_view;

selinv_status selinv_symbolic(const selinv_ctx *h, selinv_symbolic_view *v);

/* Device buffer sizes in bytes (each a multiple of 256). */
typedef struct {
  int64_t panels_bytes;  /* factor panels, batch * panel_elems scalars */
  int64_t x_bytes;       /* selected inverse, same layout */
  int64_t work_bytes;    /* device tables, normalize scratch, counters, queue */
  int64_t dtilde_bytes;  /* optional pivot blocks Dt_K (needed by selinv_backward) */
  int64_t abar_bytes;    /* adjoint / selinv_extract output on A's pattern, batch * nnz(A) scalars
                            (SELINV_LU64: batch * 2 nnz(A)) */
  int64_t trace_bytes;   /* optional selinv_trace buffer */
  int64_t tables_bytes;  /* leading part of work_bytes: the plan tables, written on upload and then only read */
} selinv_sizes_t;

selinv_status selinv_sizes(const selinv_ctx *h, selinv_sizes_t *s);

/*
 * selinv_factor -- numeric factorization and normalization.
 *   values (host): [batch][nnz(A)] in A's rowind order.
 *   panels_dev, work_dev (device, caller-owned, sizes from selinv_sizes).
 *   dtilde_dev: device buffer of dtilde_bytes or NULL (then selinv_backward
 *   is unavailable for this factorization).
 * Host: unpivoted supernodal LDL^T of every matrix of the batch (the paper
 * takes the factors from an external solver with no dynamic pivoting,
 * Section 4), then an asynchronous copy to panels_dev.  Device: the
 * normalize kernels of Alg. 1 steps 1-2 (Lhat_{C,K} = L_{C,K} L_KK^{-1},
 * Dt_K^{-1} = (L_KK D_K L_KK^T)^{-1}), which leave Dt_K^{-1} in the top s x s
 * block and Lhat_{C,K} in the bottom c x s block of each panel.
 * SELINV_LU64: unpivoted supernodal L D U (both panel sets), then
 * Lhat_{C,K} = L_{C,K} L_KK^{-1}, Uhat_{K,C}^T = U_{K,C}^T U_KK^{-T} (second
 * set) and Dt_K^{-1} = U_KK^{-1} D_K^{-1} L_KK^{-1} (first set's top block);
 * dtilde_dev must be NULL (EUNSUPPORTED otherwise).
 * Errors: SELINV_ESINGULAR on an exactly zero or non-finite pivot
 * (error_info(0) = column of B, error_info(1) = batch index).
 * Uploads the device tables into work_dev on the first call.
 */
selinv_status selinv_factor(selinv_ctx *h, const void *values, void *panels_dev, void *work_dev,
                            void *dtilde_dev, void *stream);

/*
 * selinv_normalize -- the device part of selinv_factor on its own: Alg. 1
 * steps 1-2 applied to LDL^T panels already in device memory.
 *   ldlt_dev: [batch][panel_elems] LDL^T panels (strict lower L_KK, D_K on the
 *   diagonal, L_{C,K} below), read only unless it equals panels_dev.
 *   panels_dev: receives Dt_K^{-1} (top block, full) and Lhat_{C,K}.
 *   dtilde_dev: optional Dt_K output (for selinv_backward) or NULL.
 * Asynchronous on `stream`; enables selinv_run.
 */
selinv_status selinv_normalize(selinv_ctx *h, const void *ldlt_dev, void *panels_dev, void *work_dev,
                               void *dtilde_dev, void *stream);

/*
 * selinv_factor_host -- the host part of selinv_factor only: the LDL^T
 * panels (strict lower L_KK, D_K on the diagonal, L_{C,K} below) of every
 * matrix into panels_host ([batch][panel_elems] scalars, caller-owned).  No
 * device work; does not enable selinv_run.  Errors as selinv_factor.
 */
selinv_status selinv_factor_host(selinv_ctx *h, const void *values, void *panels_host);

/*
 * selinv_factor_device -- the numeric factorization on the GPU: unpivoted
 * supernodal LDL^T of every matrix of the batch (the input the paper takes
 * from an external solver with no dynamic pivoting, Section 4), with the
 * same output as selinv_factor_host.
 *   values_dev [batch][nnz(A)] (device): A's stored lower values in rowind
 *     order (SELINV_C128: interleaved re, im).
 *   ldlt_dev [batch][panel_elems] (device, caller-owned, panels_bytes):
 *     receives the LDL^T panels (strict lower L_KK, D_K on the diagonal,
 *     L_{C,K} below); may be panels_dev, which selinv_normalize can then
 *     normalize in place.
 * Leaves to root, one launch per etree depth and step: the diagonal block's
 * LDL^T, L_KK^{-1}, L_{C,K} on FP64 MFMA, and the Schur update
 * L_{C,K} D_K L_{C,K}^T scattered into the ancestors' panels through the
 * ancestor index maps with FP64 atomic adds (the summation order of sibling
 * updates, and so the last bits, may vary between runs).  Asynchronous on
 * `stream`.  A zero or non-finite pivot is reported by the next selinv_sync
 * as SELINV_ESINGULAR (error_info(0) = column of B, error_info(1) = batch
 * index); the panels are then undefined.  selinv_logdet is valid after that
 * selinv_sync.  Uses the work buffer's tables (uploaded on the first call);
 * does not by itself enable selinv_run.
 */
selinv_status selinv_factor_device(selinv_ctx *h, const void *values_dev, void *ldlt_dev, void *work_dev,
                                   void *stream);

/*
 * selinv_run -- selected inversion (Alg. 1 second loop / Alg. 2, LDL^T form).
 * For every supernode K, root first:
 *   X_{C,K} = -X_{C,C} Lhat_{C,K};  X_KK = Dt_K^{-1} - Lhat_{C,K}^T X_{C,K};
 *   X_KK <- (X_KK + X_KK^T) / 2.
 * Reads panels_dev (normalized), writes x_dev (same layout: top block = the
 * full symmetric X_KK, bottom block = X_{C,K}).  Asynchronous on `stream`.
 * SELINV_LU64 (LU form of Alg. 1, Section 2.1): X_{C,K} = -X_{C,C} Lhat_{C,K}
 * and X_{K,C}^T = -(X_{C,C})^T Uhat_{K,C}^T, X_KK = Dt_K^{-1} - Uhat_{K,C}
 * X_{C,K} without symmetrization; the first panel set receives X_KK and
 * X_{C,K}, the second X_KK^T and X_{K,C}^T.
 * Under SELINV_SCHED_LEVELS a batch of two or more matrices runs as two
 * halves, matrices [0, ceil(batch/2)) on `stream` and the rest on a second
 * stream of the context (default priority; created with a fork and a join
 * event on the first such call, on the current device, destroyed by
 * selinv_destroy; a context used this way stays on that device, ESTATE
 * otherwise): the second stream starts after the work already enqueued on
 * `stream`, and `stream` waits for it before any later work, so the call's
 * ordering is that of a single-stream launch.  The halves touch disjoint
 * per-matrix data; the results are those of a single launch, bit for bit.
 * A single-matrix plan runs the two subtree groups below the top chain of
 * the tree (selinv_items which = 4) the same way, group 1 on `stream` and
 * group 2 on the second stream, each group's dense X_{C,C} buffers in a
 * region of their own.  A traced run (selinv_trace) keeps one stream.
 * EDEVICE when the stream or events cannot be created.
 */
selinv_status selinv_run(selinv_ctx *h, const void *panels_dev, void *x_dev, void *work_dev, void *stream);

/*
 * selinv_normalize_run -- selinv_normalize followed by selinv_run (Alg. 1
 * steps 1-2, then its second loop), with the same arguments and results, but
 * with the two overlapped under SELINV_SCHED_LEVELS: the nodes of the top
 * etree depths (those whose GEMM-1 tiles fill at most a quarter of the GPU)
 * are normalized on `stream` (their Dt^{-1} blocks on a second stream of the
 * context, at the same time as their Lhat) and their depths traversed there,
 * while the other nodes are normalized on a third stream of the context; the
 * traversal waits for that stream before its first deeper depth (the two
 * halves of a batch, as in selinv_run, each wait for it).  The two
 * streams (default priority) and four events are created on the first call,
 * on the current device, and destroyed by selinv_destroy; a context used
 * this way stays on that device (ESTATE otherwise).  Everything is ordered
 * after the work already enqueued on `stream`, and the work of the call is
 * complete when `stream` has reached it.  Under SELINV_SCHED_PERSISTENT, or
 * when the tree has no such top depths, this is the two calls in sequence.
 * Errors as selinv_normalize and selinv_run, plus EDEVICE when the stream or
 * events cannot be created.
 */
selinv_status selinv_normalize_run(selinv_ctx *h, const void *ldlt_dev, void *panels_dev, void *x_dev, void *work_dev,
                                   void *dtilde_dev, void *stream);

/*
 * selinv_normalize_run_noalloc -- for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): selinv_normalize followed by selinv_run on `stream`, with
 * the same arguments, kernels and results, but without a work buffer.  The
 * work area (plan tables, L_KK^{-1} scratch, partial products, dense X_{C,C}
 * buffers, counters) is a fixed library-owned device array of 64 MiB on each
 * GPU the library runs on, created with the library's code object and held
 * until the process ends.  The caller passes the inputs (ldlt_dev, LDL^T
 * panels) and the outputs (panels_dev, x_dev, dtilde_dev or NULL) only.
 *   Limit: plans whose forward work area exceeds 64 MiB return SELINV_ENOMEM
 *   (error_info(0) = bytes needed, error_info(1) = the limit).
 *   No hipMalloc, hipFree or other allocating routine is called.  The first
 *   call of a context on a device (and after another context used the array)
 *   copies the context's tables into the array and waits for that copy.
 *   Every call on a GPU shares that GPU's array, which keeps the last call's
 *   contents: calls that overlap on one GPU (different streams or threads)
 *   race and must be serialized by the caller.
 * Errors as selinv_normalize_run, plus SELINV_ENOMEM above.
 */
selinv_status selinv_normalize_run_noalloc(selinv_ctx *h, const void *ldlt_dev, void *panels_dev, void *x_dev,
                                           void *dtilde_dev, void *stream);

/*
 * selinv_extract -- X on A's stored lower pattern, original indexing:
 * out_dev[l][e] = (A^{-1})_{rowind[e], col(e)} of matrix l.  SELINV_LU64:
 * out_dev is [batch][2 nnz(A)], the entries as above followed by their
 * mirrors (A^{-1})_{col(e), rowind[e]}.  Asynchronous.
 */
selinv_status selinv_extract(const selinv_ctx *h, const void *x_dev, void *work_dev, void *out_dev,
                             void *stream);

/*
 * selinv_scatter -- the transpose of selinv_extract: panel_dev (panel layout,
 * [batch][panel_elems] scalars) is zeroed and vals_dev[l][e] (on A's stored
 * lower pattern, [batch][nnz(A)]) is written at the position of entry e.
 * Used to turn a gradient with respect to the extracted entries into the
 * xbar of selinv_backward.  Asynchronous on `stream`.
 */
selinv_status selinv_scatter(const selinv_ctx *h, const void *vals_dev, void *work_dev, void *panel_dev,
                             void *stream);

/*
 * selinv_backward -- adjoint of selected inversion (not in the paper; reverse
 * mode through Alg. 1 and the block LDL^T of Section 2.3).  R64 and C128; for
 * a complex-symmetric A the derivatives are holomorphic (plain transposes, no
 * conjugation): abar = dloss/da of a loss that is a holomorphic function of
 * the selected entries (a caller with a real loss of complex data conjugates
 * its cotangents on the way in and the result on the way out).
 *   xbar_dev [batch][panel_elems] (panel layout): dloss/dx for the stored
 *     selected entries (top blocks: lower triangle incl. diagonal; the strict
 *     upper triangle of every top block is ignored).  Overwritten: used as the
 *     accumulator of the reverse sweep.
 *   wlogdet_dev [batch] scalars of the context's dtype (device) or NULL:
 *     dloss/d(log det A_l) for a loss that
 *     also depends on the log-determinants (selinv_logdet).  Since
 *     d log det A / dA = A^{-1}, matrix l adds wlogdet[l] times its selected
 *     inverse on A's pattern (x2 off the diagonal) to abar.
 *   abar_dev [batch][nnz(A)]: dloss/da for A's stored lower values, original
 *     indexing (off-diagonal values stand for both (i, j) and (j, i)).
 * State: panels_dev and dtilde_dev must be the buffers the last
 * selinv_factor / selinv_normalize / selinv_normalize_run wrote (that call
 * given a dtilde_dev), and x_dev the buffer of a selinv_run (or
 * selinv_normalize_run) after it; SELINV_ESTATE otherwise.  Same work buffer.
 * Runs the level schedule (R1 leaves to root with FP64 atomic scatter-adds,
 * one per real plane, then R3 root to leaves); asynchronous on `stream`.
 * Errors: SELINV_ESTATE, SELINV_EUNSUPPORTED (context built with
 * opts.adjoint < 0), SELINV_EINVAL (null buffer).
 */
selinv_status selinv_backward(selinv_ctx *h, const void *panels_dev, const void *x_dev, const void *dtilde_dev,
                              void *xbar_dev, const void *wlogdet_dev, void *work_dev, void *abar_dev,
                              void *stream);

/*
 * selinv_check_plan -- host replay of the persistent schedule's protocol on
 * the context's tables (ready queues by depth class, dependency counters,
 * pushes).  Verifies that every work item is queued and run exactly once, no
 * queue overflows, a node starts only after its parent finished and phase 2
 * only after phase 1.  SELINV_OK or SELINV_EINVAL with a message.  Host only.
 */
selinv_status selinv_check_plan(const selinv_ctx *h);

/*
 * selinv_trace -- per-item timeline of the traversal (diagnostics).
 * trace_dev: device buffer of selinv_sizes_t.trace_bytes bytes, or NULL to
 * switch tracing off.  Each selinv_run then writes one row of eight int64
 * values per item and matrix: {item id (l * items + item), workgroup,
 * t_ticket, t_start, t_end, 0, 0, 0} in device wall-clock ticks
 * (hipDeviceAttributeWallClockRate kHz).  Persistent schedule: rows in ticket
 * order, t_ticket = when the ticket was drawn, t_start = when the item's
 * dependencies were met.  Level schedule: rows in launch order,
 * t_ticket = t_start = when the workgroup started.  The buffer is borrowed
 * until tracing is switched off; tracing slows the run slightly.
 */
selinv_status selinv_trace(selinv_ctx *h, void *trace_dev);

/*
 * selinv_items -- work items for one matrix (diagnostics).  *items receives a
 * host view of n rows of four int32 {K, type, a, b}, valid until
 * selinv_destroy.
 *   which = 0: the forward traversal's items (type: 0 GEMM-1 tile,
 *     1 diagonal-block tile, 2 single-workgroup node, 3 dense X_{C,C} gather
 *     block, 4 split-tile reduction, 5 GEMM-2 share of a tile stored by its
 *     GEMM-1 item; for type 0, b holds the column tile in its low 16 bits and
 *     the contraction part above them).  Item id i of
 *     matrix l is l * n + i in traces.
 *   which = 1: the adjoint's items in launch order (R1 leaves to root, then
 *     R3 root to leaves); type 0..11 as the BackItemType of the device plan,
 *     12 / 13 = the whole R1 / R3 of a small node in one wavefront.
 *   which = 2: the forward traversal's launches under the level and push
 *     schedules, in order: {kind (0 work items, 1 single-wavefront nodes,
 *     2 dense-buffer GEMM-1 tiles with their GEMM-2 shares, 3 push tiles,
 *     4 GEMM-1-only 128 x 128 tiles of FP64 nodes the tune table marks, 5 gathers into
 *     the dense X_{C,C} buffers, 6 GEMM-2 shares), items or records
 *     per matrix, type of the first item (-1 for push tiles), etree depth}.  The list is
 *     built for every plan; the persistent schedule does not launch by it.
 *   which = 3: the normalization chunks of selinv_normalize_run (level
 *     schedule), in order: {first level launch, its etree depth,
 *     normalization work entries of the chunk, 0}.  Chunk 0 is the top
 *     depths; the traversal of a chunk's depths waits for that chunk only.
 *   which = 4: the subtree groups of a single-matrix level plan, in launch
 *     order: {group (1 or 2), level launch, first position, end position},
 *     the positions indexing the launch list of which = 2.  From the roots
 *     down, the nodes with one child each form the top chain; the subtrees
 *     under it are dealt to two groups of about equal work, and every launch
 *     below the chain is one or more ranges of one group each.  selinv_run
 *     and selinv_normalize_run run the chain on `stream`, then group 1 there
 *     and group 2 on the context's second stream (as for the halves of a
 *     batch); empty for other plans.
 * Errors: SELINV_EINVAL for another `which`.
 */
selinv_status selinv_items(const selinv_ctx *h, int32_t which, const int32_t **items, int64_t *n);

/* log det of each matrix of the batch from the pivots (det B = prod D_jj, Section 2.3): the sum of the
   principal logarithms of the pivots.  out_host: batch doubles (R64: log |det|) or batch (re, im) pairs
   (C128).  Valid after selinv_factor or selinv_factor_host, and after selinv_factor_device once
   selinv_sync has returned; SELINV_ESTATE otherwise. */
selinv_status selinv_logdet(const selinv_ctx *h, double *out_host);

/* Wait for `stream` and report device-side errors (watchdog, HIP errors). */
selinv_status selinv_sync(selinv_ctx *h, void *stream);

const char *selinv_last_error(const selinv_ctx *h);
int64_t selinv_error_info(const selinv_ctx *h, int which);
void selinv_destroy(selinv_ctx *h);

/* Library version string. */
const char *selinv_version(void);

/* Key of this build in tune tables: "arch=<gfx target> rocm=<major.minor.patch>". */
const char *selinv_tune_key(void);

#ifdef __cplusplus
}
#endif

#endif /* SELINV_H */
