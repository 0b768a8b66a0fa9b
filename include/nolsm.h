/*
 * nolsm.h -- C ABI of the MI355X (gfx950) non-orthogonal local submatrix method.
 *
 * The library evaluates, for a batch of molecules k, the submatrix density
 *     T_k(D) = 1/2 (I - sign(T_k(S)^-1 T_k(H0) - mu I)) T_k(S)^-1      (paper, Eq. 8)
 * with a matmul-only Newton-Schulz sign iteration (Eq. 6-7), writes molecule k's
 * columns back into a density matrix that has the pattern of H0 and S (Sec. II,
 * submatrix method step 3), and reduces E = Tr(D H0) (Eq. 4) and Tr(D S).
 *
 * Conventions shared by every entry point
 *  - Pointers are DEVICE pointers unless the argument says "(host)".
 *  - The caller owns every buffer.  The library never allocates device memory:
 *    per-batch data live in a caller-provided workspace (nolsm_plan_workspace_bytes,
 *    the large per-submatrix arenas, which plans may share) and a per-plan table
 *    buffer (nolsm_plan_table_bytes: descriptors, member and tile lists, state).
 *    A plan itself is a small host object.
 *  - Work is enqueued asynchronously on `stream`; nothing synchronises the host
 *    except nolsm_check() and the first nolsm_plan_bind() of a plan to a table
 *    buffer.  Return codes report argument and launch errors only;
 *    data-dependent failures (a submatrix of S that is not positive definite, a
 *    sign iteration that did not converge) are recorded per submatrix in
 *    nolsm_stats and folded into a code by nolsm_check() after a stream sync.
 *  - nolsm_last_error() returns a thread-local message for the last non-OK return.
 *  - Calls on one plan must not overlap in time (they share its workspace).
 *
 * Matrix storage: a symmetric molecule-block-sparse matrix, compressed sparse
 * column over block columns (both triangles stored).  H0, S and D share one
 * pattern and one value layout.
 */
#ifndef NOLSM_H
#define NOLSM_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NOLSM_OK = 0,
  NOLSM_EINVAL = 1,      /* bad argument (sizes, null pointers, unbound plan)        */
  NOLSM_ENOTSPD = 2,     /* a submatrix T_k(S) is not positive definite              */
  NOLSM_ENOCONV = 3,     /* a sign iteration failed its residual test after fallback */
  NOLSM_EHIP = 4,        /* a HIP launch or runtime call failed                      */
  NOLSM_EWORKSPACE = 5,  /* workspace too small or misaligned                        */
  NOLSM_ENOMEM = 6       /* host allocation failed while planning                    */
} nolsm_status;

/* Block pattern (paper, Sec. II: the combined pattern of H0 and S).
 * blk_dim[I]   basis functions of molecule I                         [nmol]
 * blk_off[I]   first global basis function of molecule I             [nmol+1]
 * colptr[J]    stored blocks of block column J are colptr[J]..colptr[J+1]-1  [nmol+1]
 * rowblk[t]    block row of stored block t, strictly ascending within a column,
 *              and every diagonal block (J, J) is stored              [nnzb]
 * valoff[t]    offset (elements) of block t in a value array; the block is dense
 *              column major, blk_dim[rowblk[t]] x blk_dim[J]           [nnzb]
 * Value arrays of H0, S and D have nval doubles and use this layout. */
typedef struct {
  int32_t nmol;
  int64_t nnzb;
  int64_t nval;
  const int32_t *blk_dim;
  const int64_t *blk_off;
  const int64_t *colptr;
  const int32_t *rowblk;
  const int64_t *valoff;
} nolsm_pattern;

/* Form of the sign argument (Eq. 8; see nolsm_plan_options.form). */
typedef enum {
  NOLSM_FORM_SYM = 0,      /* M_k - mu I = L^-1 (H_k - mu S_k) L^-T, symmetric          */
  NOLSM_FORM_LITERAL = 1   /* A_k = S_k^-1 H_k - mu I, as Eq. 8 prints it            */
} nolsm_form;

/* Arithmetic of a sign-iteration phase. */
typedef enum {
  NOLSM_PREC_FP32 = 0,   /* FP32 operands, FP32 MFMA accumulate               */
  NOLSM_PREC_FP16 = 1,   /* FP16 operands, FP32 MFMA accumulate               */
  NOLSM_PREC_BF16 = 2    /* BF16 operands, FP32 MFMA accumulate               */
} nolsm_prec;

/* Iteration schedule for nolsm_sign_batched.
 *
 * The argument of sign() is formed in the congruent symmetric form
 *   M_k = L^-1 (H_k - mu S_k) L^-T,  S_k = L L^T (Cholesky, FP64 storage),
 * which has the spectrum of S_k^-1 H_k - mu I (Eq. 8) and gives the same density
 * in exact arithmetic: T_k(D) = 1/2 L^-T (I - sign(M_k)) L^-1 (plans of the literal
 * form iterate on S_k^-1 H_k - mu I itself, see nolsm_plan_options.form).
 * X_0 = M_k / b_k with b_k >= rho(M_k) (Gershgorin bound unless `scale` is given).
 *
 * Phases run in order.  A phase with tol > 0 stops a submatrix once
 * ||X^2 - I||_F <= tol (then runs `extra` more iterations); with
 * tol == 0 it runs exactly `iters` iterations.  A phase of order 2 (or 0) uses the
 * step
 *   X <- c1 X + c3 X X^2,  (c1, c3) = (3/2 a, -1/2 a^3)
 * with a = 1 (Newton-Schulz, Eq. 6) unless `lower` gives l_k, a lower bound on
 * min |eig(X_0)|, in which case a = sqrt(3 / (1 + l + l^2)) and l is advanced by
 * the same map each iteration (spectrum-interval scaling of Newton-Schulz).
 * A phase of order 3 uses the next member of the same polynomial family (Sec. II),
 *   X <- 1/8 X (15 I - 10 X^2 + 3 X^4),
 * which converges cubically at three products per step (two for order 2); it is
 * unscaled, so a schedule with an order-3 phase takes neither `lower` nor
 * `lower_log10` (NOLSM_EINVAL).
 *
 * After the phases, submatrices whose residual exceeds `fallback_tol` continue in
 * FP32 (at most `fallback_iters` iterations, a = 1).  Finally `panel_steps`
 * Newton-Schulz steps are applied in FP32 to the n x m panel of molecule k's own
 * columns only, and the density columns are formed in FP64. */
typedef struct {
  int32_t prec;      /* nolsm_prec */
  int32_t iters;     /* iteration count (tol == 0) or cap (tol > 0) */
  float tol;         /* convergence threshold on ||X^2 - I||_F, 0 = fixed count */
  int32_t extra;     /* iterations after reaching tol */
  int32_t order;     /* 0 or 2: Newton-Schulz; 3: the third-order polynomial step */
} nolsm_phase;

typedef struct {
  int32_t nphase;           /* 1..4 */
  nolsm_phase phase[4];
  float fallback_tol;       /* residual above which a submatrix falls back to FP32 */
  int32_t fallback_iters;   /* FP32 continuation cap (0 disables the fallback) */
  int32_t panel_steps;      /* FP32 Newton-Schulz steps on the own-column panel (>= 0) */
  const double *scale;      /* device [K] spectral bounds b_k, or NULL (Gershgorin) */
  const double *lower;      /* device [K] lower bounds l_k in (0, 1], or NULL (a = 1) */
  const float *lower_log10; /* device [K] log10 of l_k (e.g. a learned prediction), or NULL;
                               used when lower == NULL: l_k = lower_factor * 10^lower_log10[k],
                               clamped to [1e-7, 1] */
  float lower_factor;
} nolsm_schedule;

/* Per-submatrix record written by nolsm_sign_batched / nolsm_scatter_density. */
typedef struct {
  int32_t n;            /* submatrix dimension n_k */
  int32_t status;       /* 0 ok, NOLSM_ENOTSPD, NOLSM_ENOCONV */
  int32_t iters_lo;     /* iterations run in the phases */
  int32_t iters_fb;     /* FP32 fallback iterations */
  float resid;          /* last measured ||X^2 - I||_F (bounds |1 - x^2| on eig(X)) */
  int32_t fell_back;    /* 1 if the FP32 fallback ran */
  double scale;         /* b_k used */
  double tr_dh;         /* sum over molecule k's columns of D_ij H_ij (scatter) */
  double tr_ds;         /* same with S */
  float tr_x;           /* Tr(X) of the converged iterate (its eigenvalues are near +-1) */
  int32_t n_neg;        /* round((n - Tr X) / 2): eigenvalues the iteration sent to -1, i.e.
                           its count of eigenvalues of S_k^-1 H_k below mu; an independent
                           count (the inertia of H_k - mu S_k) exposes an eigenvalue that
                           converged to the wrong sign */
} nolsm_stats;

/* Where a submatrix lives inside the workspace (for inspection by tests). */
typedef struct {
  int32_t n, npad, mol, m;        /* dimension, leading dimension, first own molecule,
                                     own columns                                         */
  int32_t own_lo, nmem, ngrp, own_mem;   /* first own column, members, own molecules, the
                                     first own molecule's place in the member order      */
  int64_t off_h;                  /* bytes: M_k (FP32 npad x npad); H_k (FP64) before it
                                     with FP32 set-up products                          */
  int64_t off_s;                  /* bytes: FP64 npad x npad, S_k then L^-1 (lower)    */
  int64_t off_lo;                 /* bytes: three 4 npad^2-byte buffers: split FP16 rows
                                     of L^-1, H, U during the set-up, then the iterates */
  int64_t off_dcol;               /* bytes: FP64 npad x m density columns               */
} nolsm_sub_info;

typedef struct nolsm_plan nolsm_plan;

/* Plan a batch: the submatrices of molecules mols[0..K-1] of the pattern.
 * pattern_host must hold HOST copies of the pattern arrays.  The plan records
 * sizes, member lists and the GEMM tile work lists (host memory). */
nolsm_status nolsm_plan_create(const nolsm_pattern *pattern_host, const int32_t *mols /*host*/,
                               int32_t K, nolsm_plan **plan /*host out*/);

/* Planning options (GEMM performance depends on the submatrix size, Sec. IV-B,
 * Table II).  big_tile_min_npad: submatrices whose padded dimension is at least
 * this use the 256 x 128 FP16/BF16 tiles (two workgroups per CU), smaller ones
 * 128 x 128 tiles; a negative value selects the library default (768).  The
 * value normally comes from the autotuner's measurement of both kernels.
 * setup_products: how M_k = L^-1 T_k(H) L^-T is formed from the FP64 factor.
 * 0 (default): FP16 MFMAs on split operands (x = hi + 2^-11 lo, three partial
 * products, FP32 sums; every term within about 3 * 2^-22 of its exact value).
 * 1: FP32 operands on FP32 MFMAs.  Other values: NOLSM_EINVAL.
 * form: NOLSM_FORM_SYM (0, default) iterates on the congruent symmetric matrix
 * M_k - mu I = L^-1 (T_k(H0) - mu T_k(S)) L^-T and writes T_k(D) = 1/2 L^-T (I - X) L^-1
 * (the same T_k(D) as Eq. 8 in exact arithmetic; half of every product is formed);
 * NOLSM_FORM_LITERAL (1) evaluates Eq. 8 as printed: A_k = T_k(S)^-1 T_k(H0) - mu I
 * (S^-1 H formed in FP64), the sign iteration on the non-symmetric A_k with general
 * products (every tile), T_k(D) = 1/2 (I - sign(A_k)) T_k(S)^-1.  The literal form
 * runs every phase of a schedule in one precision and Newton-Schulz steps only
 * (nolsm_sign_batched returns NOLSM_EINVAL otherwise); it serves to check the
 * identity of the two forms and is not tuned for speed.
 * factor_tiles: the large tile products of the Cholesky factorisation of T_k(S)
 * (trailing and left-looking updates) and of L^-1 (outer block products); L and
 * L^-1 are stored in FP64 either way.  0 (default): FP32 MFMAs on operands rounded
 * to FP32 (FP32 copies of the panels, in the iteration arena during the set-up),
 * FP32 sums (L^-1 S L^-T - I of a few 1e-7, density columns within about 1e-7 of
 * the FP64 factor's).  1: FP64 MFMAs throughout.  Other values: NOLSM_EINVAL. */
typedef struct {
  int32_t big_tile_min_npad;
  int32_t setup_products;
  int32_t persist;                /* 0 (default): every arena in the workspace.  1: the
                                     set-up results M_k and L^-1 of every submatrix live in
                                     a buffer of their own (nolsm_plan_persist_bytes, bound
                                     with nolsm_plan_bind_persist), so they survive while
                                     other plans use the shared workspace; a chemical-
                                     potential search then sets each batch up once.     */
  int32_t factor_tiles;
  int32_t form;                   /* nolsm_form */
  int32_t reserved[3];            /* must be zero */
} nolsm_plan_options;

/* nolsm_plan_create with options (host pointer; NULL = defaults).
 * NOLSM_EINVAL if a reserved field is non-zero. */
nolsm_status nolsm_plan_create_ex(const nolsm_pattern *pattern_host, const int32_t *mols /*host*/,
                                  int32_t K, const nolsm_plan_options *options /*host*/,
                                  nolsm_plan **plan /*host out*/);
/* Plan a batch of combined submatrices (Sec. IV-B: columns are combined so that one
 * submatrix serves several of them): submatrix g serves the block columns of the
 * molecules grp_mols[grp_ptr[g] .. grp_ptr[g+1]-1] (host arrays; grp_ptr[0] = 0).
 * Its rows are the union of those block columns' stored rows; a group of several
 * molecules puts them first (ascending) and the other rows after them (ascending),
 * a single molecule keeps the ascending order of nolsm_plan_create, which is this
 * call with one molecule per group.  Each molecule may appear once.  Limits per
 * submatrix: 1,024 member molecules, n <= 8,192 (NOLSM_EINVAL). */
nolsm_status nolsm_plan_create_groups(const nolsm_pattern *pattern_host, const int32_t *grp_ptr,
                                      const int32_t *grp_mols, int32_t ngroups,
                                      const nolsm_plan_options *options /*host, nullable*/,
                                      nolsm_plan **plan /*host out*/);

/* Performance-aware submatrix combination (Sec. IV-B, Eq. 9 and Eq. 10), host only.
 * Starting from one group per molecule of mols[0..K-1], repeatedly combine the two
 * groups with the largest gain cost(n_i) + cost(n_j) - cost(n_i + n_j - n_ij) among
 * the pairs whose submatrices share a row (n_ij > 0: the functions of the shared
 * rows), until no pair gains.  cost(n) = n^3 (criterion 9, the flops of the dense
 * products) or n^3 / rate(n) (criterion 10, their predicted run time), with rate(n)
 * interpolated linearly in the measured table (rate_n ascending, clamped at its
 * ends).  Ties go to the pair whose smallest molecules, smaller first, come first.
 * Pairs whose combined n would exceed max_n (> 0) are not combined.
 * Output: ngroups_out groups in grp_ptr [K+1] / grp_mols [K] (host, caller
 * allocated), each ascending, ordered by first molecule.
 * NOLSM_EINVAL for bad arguments (criterion, table not ascending or not positive,
 * molecules out of range or repeated). */
typedef struct {
  int32_t criterion;        /* 9 or 10 */
  int32_t max_n;            /* 0 = no limit */
  int32_t npoints;          /* rows of the rate table (criterion 10), >= 1 */
  int32_t pad;
  const double *rate_n;     /* host [npoints] dimensions, strictly ascending */
  const double *rate;       /* host [npoints] throughput at those dimensions (> 0) */
} nolsm_combine_options;

nolsm_status nolsm_combine(const nolsm_pattern *pattern_host, const int32_t *mols /*host*/,
                           int32_t K, const nolsm_combine_options *options /*host*/,
                           int32_t *grp_ptr /*host out [K+1]*/, int32_t *grp_mols /*host out [K]*/,
                           int32_t *ngroups_out /*host out*/);

void nolsm_plan_destroy(nolsm_plan *plan);

/* Device workspace bytes the plan needs: a 256-byte header shared by every plan
 * bound to the same workspace, then the per-submatrix arenas (256-byte aligned
 * base required). */
size_t nolsm_plan_workspace_bytes(const nolsm_plan *plan);

/* Device table-buffer bytes of the plan (descriptors, member lists, GEMM tile
 * lists, per-submatrix state); one buffer per plan, 256-byte aligned. */
size_t nolsm_plan_table_bytes(const nolsm_plan *plan);

/* Attach the plan to its table buffer and to a workspace.  The first bind to a
 * given table buffer uploads the tables and clears the state on `stream` and
 * then synchronises the stream (the host copies must outlive the upload); later
 * binds with the same table buffer do no device work at all, so several plans can
 * take turns on one workspace inside stream capture (a HIP graph of a whole
 * multi-batch step).  Calls on plans sharing a workspace must not overlap.
 * Errors: NOLSM_EINVAL for null pointers, NOLSM_EWORKSPACE for buffers that are
 * too small or misaligned, NOLSM_EHIP for a failed upload. */
nolsm_status nolsm_plan_bind(nolsm_plan *plan, void *tables, size_t table_bytes, void *workspace,
                             size_t bytes, hipStream_t stream);

/* Bytes of the plan's own set-up buffer (256-byte aligned base required): M_k
 * (FP32) and L^-1 (FP64) of every submatrix; 0 unless the plan was created with
 * persist = 1. */
size_t nolsm_plan_persist_bytes(const nolsm_plan *plan);

/* nolsm_plan_bind for a plan created with persist = 1 (NOLSM_EINVAL otherwise, and
 * nolsm_plan_bind refuses such a plan): `persist` (persist_bytes) holds this plan's
 * set-up results and must not be shared with another plan; `workspace` may be.
 * While the plan keeps the same table buffer and persist buffer, rebinding keeps
 * its set-up (and the Gershgorin bounds of nolsm_features) current, so a later
 * nolsm_sign_batched needs no new gather or set-up.  Binding with a different
 * workspace or persist buffer than the last time re-uploads the descriptors and
 * synchronises `stream` (not capturable); the same pair again does no device work. */
nolsm_status nolsm_plan_bind_persist(nolsm_plan *plan, void *tables, size_t table_bytes,
                                     void *workspace, size_t bytes, void *persist,
                                     size_t persist_bytes, hipStream_t stream);

/* Layout of submatrix i (0 <= i < K) inside the bound workspace (off_h and off_s
 * inside the persist buffer for a plan created with persist = 1). */
nolsm_status nolsm_plan_query(const nolsm_plan *plan, int32_t i, nolsm_sub_info *info /*host*/);

/* Step 1 of the submatrix method for H0 and S (Sec. II; Eq. 8 builds both from the
 * combined pattern): for every planned molecule k, gather the dense principal
 * submatrices T_k(H0), T_k(S) (FP64, column major) on the functions of the
 * molecules stored in block column k, in ascending molecule order.  Blocks absent
 * from the pattern are zero.  pattern_dev holds DEVICE copies of the arrays. */
nolsm_status nolsm_build_submatrices(nolsm_plan *plan, const nolsm_pattern *pattern_dev,
                                     const double *H_val, const double *S_val,
                                     hipStream_t stream);

/* The mu-independent part of step 2 alone: FP64 Cholesky T_k(S) = L L^T, L^-1 and
 * M_k = L^-1 T_k(H0) L^-T for every planned submatrix.  A following
 * nolsm_sign_batched (for any mu) reuses it instead of repeating it, until the
 * next nolsm_build_submatrices; this is how a chemical-potential search shares
 * one set-up between its mu values, since the argument is M_k - mu I. */
nolsm_status nolsm_setup_batched(nolsm_plan *plan, hipStream_t stream);

/* Per-submatrix descriptors of A_k = M_k - mu I for the learned schedule
 * (requires the set-up; runs it if needed).  feat: device [K * NOLSM_NFEAT] FP32,
 * row k = (log n, members/100, m/32, log b, Gershgorin lower and upper edge / b,
 * Tr A/(n b), ||A||_F/(sqrt(n) b), std diag/b, min|A_ii|/b, mean and max
 * off-diagonal row sum / b, fraction of negative diagonal entries,
 * mean|A_ii|/b, min|A_ii| / (||A||_F/sqrt(n)), 1), with b the Gershgorin bound.
 * The bounds b also stay in the plan's state: a following nolsm_sign_batched with
 * the same mu (and no new gather or set-up in between) scales by them instead of
 * making its own pass over M_k. */
#define NOLSM_NFEAT 16
nolsm_status nolsm_features(nolsm_plan *plan, double mu, float *feat, hipStream_t stream);

/* Step 2 (Eq. 8 via Eq. 6-7): FP64 Cholesky and transform, scaling, the batched
 * sign iteration under `sched` (NULL = plain FP32 Newton-Schulz to convergence),
 * the FP32 fallback and the own-column panel refinement, and the FP64 density
 * columns T_k(D)[:, own columns].  stats: device [K] (may be NULL).
 * NOLSM_EINVAL, with nothing enqueued: a null plan, a non-finite mu, a bad
 * schedule (nphase outside 1..4, a phase with an unknown precision, iters outside
 * 0..1000, negative extra or tol, an order other than 0, 2 or 3, an order-3 phase
 * with lower bounds, panel_steps outside 0..2, fallback_iters outside 0..1000),
 * checked in that order, then an unbound plan. */
nolsm_status nolsm_sign_batched(nolsm_plan *plan, double mu, const nolsm_schedule *sched /*host*/,
                                nolsm_stats *stats, hipStream_t stream);

/* Step 3 (Sec. II): write molecule k's density columns into block column k of D
 * (same pattern and layout as H0, S) -- every molecule of a combined submatrix from
 * that submatrix -- and record the submatrix's own columns' contribution to
 * Tr(D H0) and Tr(D S) in stats[i].tr_dh / tr_ds.  Only block columns of planned
 * molecules are written. */
nolsm_status nolsm_scatter_density(nolsm_plan *plan, const nolsm_pattern *pattern_dev,
                                   double *D_val, const double *H_val, const double *S_val,
                                   nolsm_stats *stats, hipStream_t stream);

/* Eq. 4 and the electron count: out2[0] = Tr(D H0) = sum_ij D_ij H0_ij (H0 is
 * symmetric), out2[1] = Tr(D S).  col_traces: device [2*nmol] scratch that
 * receives the per-block-column sums; the final sum runs over block columns in
 * ascending order, so the result is bitwise reproducible. */
nolsm_status nolsm_energy(const nolsm_pattern *pattern_dev, int32_t nmol, const double *D_val,
                          const double *H_val, const double *S_val, double *col_traces,
                          double *out2, hipStream_t stream);

/* nolsm_energy for callers that cannot allocate or pass scratch memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation): the
 * same result, bit for bit, with the per-block-column sums kept in a fixed device
 * array of the library (2 * NOLSM_ENERGY_NOALLOC_MAXMOL doubles, 2 MiB, one copy
 * per GPU, held until the process ends).  Allocates nothing.  Every call on one GPU
 * uses that GPU's array, so calls that overlap in time on one GPU (several streams
 * or threads) race; the array keeps the last call's sums.
 * NOLSM_EINVAL for a bad argument or nmol > NOLSM_ENERGY_NOALLOC_MAXMOL;
 * NOLSM_EHIP if the array's address cannot be obtained or a launch fails. */
#define NOLSM_ENERGY_NOALLOC_MAXMOL 131072
nolsm_status nolsm_energy_noalloc(const nolsm_pattern *pattern_dev, int32_t nmol,
                                  const double *D_val, const double *H_val, const double *S_val,
                                  double *out2, hipStream_t stream);

/* Learned schedule: a multilayer perceptron NOLSM_NFEAT -> 64 -> 64 -> nout
 * (SiLU hidden activations, linear output, FP32) with hand-written training
 * kernels.  Parameters are one FP32 array, in order W1[64][16], b1[64],
 * W2[64][64], b2[64], W3[nout][64], b3[nout] (row major, y = W x + b).
 * x: [B][16], y and targets: [B][nout], all row major, device memory.
 * Reductions over the batch run in a fixed order (bitwise reproducible). */
#define NOLSM_MLP_HIDDEN 64
#define NOLSM_MLP_MAXOUT 4
int64_t nolsm_mlp_param_count(int32_t nout);
/* Device scratch floats needed by nolsm_mlp_backward / nolsm_mlp_mse for batch B. */
int64_t nolsm_mlp_scratch_floats(int64_t B, int32_t nout);

/* y = MLP(x).  act (nullable): [B][2*64] pre-activations saved for the backward. */
nolsm_status nolsm_mlp_forward(const float *params, int32_t nout, const float *x, int64_t B,
                               float *y, float *act, hipStream_t stream);
/* grad = d(loss)/d(params) given dy = d(loss)/dy and the saved pre-activations. */
nolsm_status nolsm_mlp_backward(const float *params, int32_t nout, const float *x,
                                const float *act, const float *dy, int64_t B, float *grad,
                                float *scratch, hipStream_t stream);
/* Mean squared error over the batch: loss[0] = sum (y - t)^2 / (B nout), dy = its gradient. */
nolsm_status nolsm_mlp_mse(const float *y, const float *t, int64_t B, int32_t nout, float *dy,
                           float *loss, float *scratch, hipStream_t stream);
/* One Adam step (Kingma and Ba, 2015) with bias correction; step counts from 1. */
nolsm_status nolsm_mlp_adam(float *params, const float *grad, float *m, float *v, int64_t P,
                            float lr, float beta1, float beta2, float eps, int32_t step,
                            hipStream_t stream);

/* Measurement (not needed for results).  With timing enabled, the plan records a
 * pair of HIP events on `stream` around every launch group below, and
 * nolsm_plan_get_timings() (which synchronises on those events) returns the
 * accumulated milliseconds since the last reset.  The sign-iteration GEMM launches
 * are timed one by one, so ms_gemm / n_gemm is their average duration. */
typedef struct {
  double ms_gather;      /* nolsm_build_submatrices                                  */
  double ms_setup;       /* FP64 Cholesky, inverse and transform                     */
  double ms_sign;        /* scaling and every sign-iteration launch (incl. GEMMs)    */
  double ms_gemm;        /* sign-iteration GEMM launches only                        */
  double ms_panel;       /* panel refinement and density columns                     */
  double ms_scatter;     /* nolsm_scatter_density                                    */
  int64_t n_gemm;        /* GEMM launches timed                                      */
  double gemm_flop;      /* executed MFMA flops of the tiles that were active (device count) */
} nolsm_timings;

/* gemm_flop comes from a counter in the first 256 bytes of the workspace, shared by
 * every plan bound to that workspace: it accumulates over all of them and is
 * cleared by a call with reset != 0 (it starts undefined). */
nolsm_status nolsm_plan_set_timing(nolsm_plan *plan, int enable);
nolsm_status nolsm_plan_get_timings(nolsm_plan *plan, nolsm_timings *out /*host*/, int reset);

/* Chemical-potential search (Sec. V-A: the runs iterate mu until the system is
 * charge neutral).  Host-side bisection of the electron count N(mu) = Tr(D(mu) S)
 * against n_target: the caller evaluates N at s.mu (nolsm_sign_batched and
 * nolsm_scatter_density for every batch at that mu, then nolsm_energy) and passes
 * it to nolsm_mu_search_update, until s.done != 0.  The bracket keeps N(lo) below
 * n_target - tol and N(hi) above n_target + tol (the initial [mu_lo, mu_hi] is
 * taken as such); each trial is the bracket's midpoint; the search ends at the
 * first trial with |N - n_target| <= tol (done = 1, s.mu is that trial) or after
 * max_iter trials (done = -1, s.mu is the last trial).  Every trial shares the
 * set-up M_k = L^-1 H_k L^-T, since the argument of sign() is M_k - mu I. */
typedef struct {
  double n_target, tol;   /* electron count sought, accepted deviation           */
  double lo, hi;          /* current bracket                                      */
  double mu;              /* trial to evaluate next; the result once done != 0    */
  double last_n;          /* N at the last evaluated trial                        */
  int32_t iters;          /* trials evaluated                                     */
  int32_t max_iter;       /* 1..1000                                              */
  int32_t done;           /* 0 searching, 1 converged, -1 max_iter reached        */
  int32_t pad;
} nolsm_mu_search;

/* NOLSM_EINVAL for a null pointer, non-finite values, mu_lo >= mu_hi, tol < 0 or
 * max_iter outside 1..1000. */
nolsm_status nolsm_mu_search_init(nolsm_mu_search *s /*host*/, double n_target, double mu_lo,
                                  double mu_hi, double tol, int32_t max_iter);
/* Fold N(s->mu) into the bracket and set the next trial.  NOLSM_EINVAL for a null
 * pointer, a non-finite count or a search that has already ended. */
nolsm_status nolsm_mu_search_update(nolsm_mu_search *s /*host*/, double n_at_mu);

/* Synchronise `stream`, read the plan's device status words, and return
 * NOLSM_ENOTSPD / NOLSM_ENOCONV if any submatrix failed (else NOLSM_OK). */
nolsm_status nolsm_check(nolsm_plan *plan, hipStream_t stream);

const char *nolsm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* NOLSM_H */
