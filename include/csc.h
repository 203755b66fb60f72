/*
 * csc.h -- C ABI of libcsc: compressive spectral clustering of static and dynamic graphs
 * on one AMD Instinct MI355X (gfx950).
 *
 * The calls follow the statement of the problem in Martin, Loukas and Vandergheynst,
 * "Fast Approximate Spectral Clustering for Dynamic Networks" (ICML 2017): a graph
 * sequence G_1..G_tau, a reuse fraction p and a number of random signals d give one
 * assignment per snapshot (Algorithm 1, Sec. 4.1), built on polynomial filtering of
 * random signals (Sec. 2.2, Step 1) with a cut-off found by eigencount (Sec. 3.2).
 *
 * Conventions shared by every call
 *  - Every call returns csc_status; nothing throws across the ABI.  csc_last_error()
 *    returns a thread-local message describing the last failure.
 *  - "device" pointers are HIP device allocations owned by the caller; the library never
 *    frees them.  "host" pointers are ordinary host memory.
 *  - Work is enqueued on the caller's hipStream_t, passed as void* (NULL = the null
 *    stream).  Calls documented as "synchronising" wait for that stream before returning
 *    host results; all others are asynchronous.
 *  - Dense blocks are row-major: element (i, j) of an n x w block X with leading
 *    dimension ldx (in elements, ldx >= w) is X[i * ldx + j].
 *  - Handles (csc_graph, csc_dyn) own their internal device memory, allocated in
 *    *_create.  The exceptions say so where they are declared: csc_lmax and
 *    csc_graph_distance take temporary memory, and a dynamic state that tracks similarity
 *    allocates its copy of the previous operator on the first snapshot (and grows it for a
 *    larger one).  Scratch memory of the other calls comes from a caller buffer `work`
 *    whose size is given by the matching *_workspace_bytes query; a too-small buffer is
 *    CSC_E_ARG.
 *  - Results are deterministic given the inputs and seeds: every floating-point
 *    reduction runs in a fixed order.  The one floating-point atomic sum (duplicate draws
 *    in compressive k-means) adds identical values, so its result does not depend on the
 *    order either.
 */
#ifndef CSC_H
#define CSC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CSC_OK = 0,
  CSC_E_ARG = 1,    /* invalid argument (size, range, alignment, aliasing, workspace) */
  CSC_E_GRAPH = 2,  /* the CSR input is not a simple symmetric graph with w > 0 */
  CSC_E_DTYPE = 3,  /* unsupported element type for this argument */
  CSC_E_NOMEM = 4,  /* device allocation failed (in *_create, or where a call says it allocates) */
  CSC_E_HIP = 5,    /* a HIP runtime call failed */
  CSC_E_STATE = 6   /* handle used out of order */
} csc_status;

/* Iterate storage modes (the iter_dt arguments only):
 *  - CSC_F16: the Chebyshev iterates are stored in IEEE binary16 (11 significant bits
 *    against BF16's 8, at the same two bytes).  The iterates of the filter satisfy
 *    |Z_j[:, c]|_2 <= |X[:, c]|_2 (|T_j| <= 1 on the mapped spectrum), so every entry stays
 *    inside binary16's range when every column of X has 2-norm below 2^15; the caller
 *    guarantees that (signals of variance 1/d on n nodes have column norms sqrt(n / d)).
 *    Entries below 2^-14 are stored as binary16 subnormals (absolute spacing 2^-24).
 *  - CSC_BF16S / CSC_F16S: BF16 / binary16 copies of the iterates serve the neighbour
 *    gathers and the kept basis, while the three-term recurrence itself is carried in FP32
 *    (its state is never rounded). */
typedef enum {
  CSC_F32 = 0,
  CSC_BF16 = 1,
  CSC_F64 = 2,
  CSC_BF16S = 3,
  CSC_F16 = 4,
  CSC_F16S = 5
} csc_dtype;

typedef enum { CSC_DAMP_NONE = 0, CSC_DAMP_JACKSON = 1 } csc_damping;

/* The two Laplacians of Sec. 2.1: normalized L = I - D^{-1/2} W D^{-1/2}, spectrum in
 * [0, 2]; combinatorial L = D - W, spectrum in [0, max over edges (i, j) of d_i + d_j]. */
typedef enum { CSC_LAP_NORMALIZED = 0, CSC_LAP_COMBINATORIAL = 1 } csc_laplacian;

typedef struct csc_graph_s* csc_graph;
typedef struct csc_dyn_s* csc_dyn;

/* Thread-local description of the last error (never NULL). */
const char* csc_last_error(void);
/* Library version, major * 10000 + minor * 100 + patch. */
int csc_version(void);

/* ---------------------------------------------------------------------------------
 * Graph operator (Sec. 2.1).  From the symmetric weight matrix W in CSR form, builds on
 * the device either
 *  - lap = CSC_LAP_NORMALIZED: the normalized adjacency A = D^{-1/2} W D^{-1/2}, so that
 *    L = I - A.  An isolated node (degree 0) gets D^{-1/2} = 0, i.e. an identity row in L
 *    and eigenvalue 1; or
 *  - lap = CSC_LAP_COMBINATORIAL: W itself and the degrees D, so that L = D - W (an
 *    isolated node is a zero row, eigenvalue 0).  The spectrum bound of csc_lmax is
 *    computed here, so create and update synchronise `stream` for such a graph.
 * The number of isolated nodes is reported by csc_graph_info.
 *
 * rowptr_d: device int64[n + 1]; colidx_d: device int32[nnz], sorted strictly increasing
 * within each row; w_d: device double[nnz], all > 0.  No self-loops; W symmetric (entry
 * (i, j) present with the same weight as (j, i)).  With validate != 0 every one of these
 * properties is checked on the device and a violation returns CSC_E_GRAPH (the call then
 * synchronises `stream`); with validate == 0 the caller guarantees them.
 * val_dt: storage type of A's values (CSC_F32 or CSC_BF16).  nnz_capacity >= nnz sizes
 * the handle so that csc_graph_update can later load a graph with up to that many
 * entries without allocating.  The handle copies what it needs; the inputs may be freed
 * once `stream` has passed the call.
 */
csc_status csc_graph_create(int64_t n, int64_t nnz, int64_t nnz_capacity,
                            const int64_t* rowptr_d, const int32_t* colidx_d,
                            const double* w_d, csc_dtype val_dt, csc_laplacian lap,
                            int validate, void* stream, csc_graph* out);
/* Rebuild the operator of an existing handle from a new W with the same n and
 * nnz <= nnz_capacity (a new snapshot of a dynamic graph).  Allocates nothing. */
csc_status csc_graph_update(csc_graph g, int64_t nnz, const int64_t* rowptr_d,
                            const int32_t* colidx_d, const double* w_d, int validate,
                            void* stream);
csc_status csc_graph_destroy(csc_graph g);
/* Sizes and the number of isolated nodes (synchronising). */
csc_status csc_graph_info(csc_graph g, int64_t* n, int64_t* nnz, int64_t* isolated);
/* Device views of the operator: int32 row pointers (n + 1), int32 column indices, A's
 * values (type *val_dt), D^{-1/2} as double[n], and for every entry e = (i, j) the index
 * of its mirror entry (j, i).  Valid until the next update or destroy. */
csc_status csc_graph_arrays(csc_graph g, const int32_t** rowptr, const int32_t** colidx,
                            void** vals, csc_dtype* val_dt, const double** dinv,
                            const int32_t** mirror);

/* Upper bound of the spectrum of L used to map [0, lmax] onto [-1, 1] (Sec. 3.2 gives
 * none).  iters == 0 returns the graph's fixed bound: 2 for the normalized Laplacian; for
 * the combinatorial one, max over stored entries (i, j) of d_i + d_j (Anderson and Morley,
 * 1985), computed in FP64, or 1 for a graph without edges.  iters > 0 runs that many power
 * iterations on L from a fixed pseudo-random start and returns 1.01 (rho + r), clamped to
 * at most the fixed bound, where rho is the last Rayleigh quotient and r the norm of its
 * residual L x - rho x (|x| = 1).  Allocates temporary device memory.  Synchronising. */
csc_status csc_lmax(csc_graph g, int iters, double* lmax, void* stream);

/* Edge similarity of two snapshots (Sec. 4, the metrics of graph similarity):
 * *rho = ||L(g2) - L(g1)||_F, summed in FP64 over the union of the two sparsity patterns
 * from the stored values (plus the degrees for L = D - W).  Both graphs must have the same
 * n and Laplacian kind (CSC_E_ARG otherwise).  With BF16 values the result carries their
 * rounding.  Allocates temporary device memory.  Synchronising. */
csc_status csc_graph_distance(csc_graph g1, csc_graph g2, double* rho, void* stream);

/* ---------------------------------------------------------------------------------
 * Chebyshev coefficients of the ideal low-pass (Sec. 3.2): h(lambda) = sum_{j=0..m}
 * a[j] T_j(2 lambda / lmax - 1) approximates the step 1[lambda <= lambda_c] of the
 * ideal filter H_k (eq. Hk): a[0] = 1 - theta_c / pi and a[j] = -2 sin(j theta_c) /
 * (j pi) with theta_c = arccos(2 lambda_c / lmax - 1), each multiplied by the Jackson
 * factor when damp == CSC_DAMP_JACKSON.  a: host double[m + 1].  Host only.
 */
csc_status csc_cheb_coeffs(int m, double lmax, double lambda_c, csc_damping damp, double* a);

/* ---------------------------------------------------------------------------------
 * Chebyshev filtering of a block of signals (Sec. 2.2, Step 1, and Sec. 3.2):
 *     Y = sum_{j=0..m} a[j] T_j(L~) X,  L~ = (2 / lmax) L - I,
 * by the three-term recurrence Z_0 = X, Z_1 = L~ X, Z_{j+1} = 2 L~ Z_j - Z_{j-1}, each
 * step one fused kernel (sparse product, recurrence and coefficient accumulation).
 *
 * X: device n x w block, type x_dt (F32/BF16/F64), leading dimension ldx.
 * Y: device n x w block, type y_dt (F32/BF16/F64), leading dimension ldy; must not
 *    overlap X.  a: host double[m + 1].  iter_dt: storage of the iterates Z_j: CSC_F32;
 *    CSC_BF16 or CSC_F16 (rounded to BF16 / binary16 at every step, half the traffic;
 *    binary16 keeps 3 more bits, within the range condition stated with csc_dtype); or
 *    CSC_BF16S / CSC_F16S (BF16 / binary16 copies for the gathers, FP32 recurrence state).
 *    Arithmetic is always FP32.
 * moments: NULL, or device double[m + 1] receiving mu_j = <X, T_j(L~) X> (summed over the
 *    w columns) for j = 0..m, obtained during the same pass from the doubling identities
 *    T_j^2 = (T_2j + T_0) / 2 and T_{j+1} T_j = (T_2j+1 + T_1) / 2.
 * work: device scratch of csc_cheb_filter_workspace_bytes(n, w, iter_dt) bytes.
 * Asynchronous.
 */
size_t csc_cheb_filter_workspace_bytes(int64_t n, int w, csc_dtype iter_dt);
csc_status csc_cheb_filter(csc_graph g, double lmax, int m, const double* a, const void* X,
                           csc_dtype x_dt, int64_t ldx, void* Y, csc_dtype y_dt, int64_t ldy,
                           int w, csc_dtype iter_dt, double* moments, void* work,
                           size_t work_bytes, void* stream);

/* Chebyshev moments only: mu_j = <P, T_j(L~) P> for j = 0..m (device double[m + 1]) from
 * floor(m / 2) + 1 operator products (doubling).  m >= 1.  Asynchronous. */
csc_status csc_cheb_moments(csc_graph g, double lmax, int m, const void* P, csc_dtype p_dt,
                            int64_t ldp, int n_probe, csc_dtype iter_dt, double* moments,
                            void* work, size_t work_bytes, void* stream);

/* ---------------------------------------------------------------------------------
 * Eigencount and dichotomy for the cut-off (Sec. 3.2; Sec. 4.1).  The count below a
 * cut-off lambda is Hutchinson's estimate c(lambda) = sum_j a_j(lambda) mu_j /
 * (sigma2 * n_probe) with mu the Chebyshev moments of the probes P (n x n_probe, i.i.d.
 * entries of variance sigma2).  The dichotomy runs n_cand fixed steps on [lo, hi]:
 * mid = (lo + hi) / 2, lo = mid when c(mid) < k, else hi = mid; it returns
 * *lambda_c = hi and *count = c(hi).  trace (host double[2 * n_cand] or NULL) receives
 * (mid, c(mid)) per step; moments_out (host double[m + 1] or NULL) the moments.
 * One device pass over the probes, then host FP64 arithmetic.  Synchronising.
 */
csc_status csc_eigcount(csc_graph g, double lmax, int m, csc_damping damp, const void* P,
                        csc_dtype p_dt, int64_t ldp, int n_probe, double sigma2, double k,
                        int n_cand, double lo, double hi, csc_dtype iter_dt,
                        double* lambda_c, double* count, double* trace,
                        double* moments_out, void* work, size_t work_bytes, void* stream);
/* The host half of csc_eigcount, from moments already on the host.  Host only. */
csc_status csc_eigcount_from_moments(const double* mu, int m, double lmax, csc_damping damp,
                                     double sigma2, int n_probe, double k, int n_cand,
                                     double lo, double hi, double* lambda_c, double* count,
                                     double* trace);

/* <X, Y> over an n x w block pair in FP64 with a fixed reduction order (device double[1]
 * result).  Used for the eigencount of filtered signals, c = <P, h(L) P> / (sigma2 w).
 * work: csc_dot_workspace_bytes(n).  Asynchronous. */
size_t csc_dot_workspace_bytes(int64_t n);
csc_status csc_dot(const void* X, csc_dtype x_dt, int64_t ldx, const void* Y, csc_dtype y_dt,
                   int64_t ldy, int64_t n, int w, double* result, void* work,
                   size_t work_bytes, void* stream);

/* ---------------------------------------------------------------------------------
 * Random signals (Sec. 2.2): X (device n x w, type dt, leading dimension ldx) gets
 * i.i.d. N(0, sigma^2) entries from Philox4x32-10 (Salmon et al., SC 2011): for row i and
 * column pair q the counter is (i, q, stream_id_lo, stream_id_hi) and the key
 * (seed_lo, seed_hi); the four output words give two 53-bit uniforms u1, u2 in (0, 1)
 * and Box-Muller gives columns 2q and 2q + 1 (FP64, rounded once).  row0 offsets the
 * row index (to draw a slice of a larger block).  Asynchronous.
 */
csc_status csc_randn(void* X, csc_dtype dt, int64_t n, int w, int64_t ldx, int64_t row0,
                     uint64_t seed, uint64_t stream_id, double sigma, void* stream);
/* count uniforms in (0, 1) of (seed, stream_id): counter (j, 0, stream lo, stream hi).
 * u: device double[count].  Asynchronous. */
csc_status csc_uniforms(double* u, int count, uint64_t seed, uint64_t stream_id,
                        void* stream);

/* ---------------------------------------------------------------------------------
 * k-means on the rows of the features (Sec. 2.1, eq. SC_cost).
 *
 * csc_kmeans_assign: labels[i] = argmin_c sum_t (F[i, t] - C[c, t])^2 for the n rows of
 * F (device, type f_dt, leading dimension ldf, d columns) and the k centroids C (device
 * float[k * d], row-major).  For d <= 256 and 16-byte aligned rows the scores
 * ||C_c||^2 - 2 F_i.C_c are formed on the matrix cores from two BF16 parts of C (hi, mid;
 * the rest, R_c, within 2^-16 of each value) and exact BF16 splits of FP32 rows (three parts;
 * BF16 rows are exact): each pair of 32-column steps' leading products goes to a fresh FP32
 * accumulator, the pairs are summed in FP32, and the small cross products to a second FP32
 * sum; the score and its interval are formed in FP32, with a half-width of
 * (2 * 72 + 16) * 2^-24 ||F_i|| ||C_c|| + 2 ||F_i|| ||R_c|| + 8 * 2^-24 ||C_c||^2 + 2^-110
 * that covers the dropped part and every rounding.  A row with one centroid whose interval can hold the
 * minimum is decided; with two, both are re-scored in the FP64 direct form; with more, every
 * centroid is.  Rows that are not 16-byte aligned take a vector path instead: candidates are
 * ranked in FP32 and the two best re-scored in FP64.  Exact ties go to the lowest index.
 * Every k-means call takes 1 <= d <= 256 columns and 1 <= k <= 240 centroids (CSC_E_ARG
 * otherwise, before any device memory is touched).  labels: device
 * int32[n]; best_d2: device float[n] (the FP64 squared distance to the chosen centroid,
 * rounded) or NULL.  sums (device float[k * d]) and counts (device int32[k]), each
 * optional: the Lloyd partial sums of the new assignment, sums[c] = the sum of the rows
 * labelled c (accumulated in 64-bit fixed point, exact up to the fixed-point scale, then
 * rounded once to FP32) and counts[c] their number; they take a second pass over F.  work:
 * csc_kmeans_workspace_bytes(n, d, k) bytes (the split centroids and the sums live there).
 * Asynchronous.
 *
 * csc_kmeans_update: C[c] = mean of the rows labelled c; an empty cluster keeps its
 * previous centroid (C is read and overwritten); rows whose label is outside [0, k) are
 * ignored; counts: device int32[k] or NULL.  Sums in 64-bit fixed point: each value is
 * rounded (half to even) to an integer multiple of 2^-S, S = 62 - e - ceil(log2 n) (kept
 * within [-60, 120]) for max |F| < 2^e, and the integers are added exactly, so the result
 * does not depend on the order of the rows (bit-reproducible).  The rows are ordered by
 * label (counting sort) and summed in chunks of one label.  n < 2^31 (CSC_E_ARG
 * otherwise).  work: csc_kmeans_workspace_bytes(n, d, k) (it also holds the row order and
 * the chunk sums).  Asynchronous.
 *
 * csc_kmeans_seed: k-means++ (Arthur and Vassilvitskii, 2007) driven by the device
 * uniforms u[0..k-1]: the first centre is row floor(u[0] n); centre j is the first row
 * whose running sum of squared distances (FP64) to the chosen centres exceeds u[j] times
 * their total.  Writes C (device float[k * d]) and idx (device int32[k] or NULL).
 * Asynchronous.
 *
 * csc_kmeans: seeding (init == 0, uniforms of (seed, stream_id)) or the given C
 * (init == 1), then `iters` rounds of assign + update and a final assignment.
 * objective: host double[iters + 1] or NULL (sum of squared distances of each assignment;
 * synchronising when given).
 */
size_t csc_kmeans_workspace_bytes(int64_t n, int d, int k);
csc_status csc_kmeans_assign(const void* F, csc_dtype f_dt, int64_t ldf, int64_t n, int d,
                             const float* C, int k, int32_t* labels, float* best_d2,
                             float* sums, int32_t* counts, void* work, size_t work_bytes,
                             void* stream);
/* csc_kmeans_assign_noalloc: for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc), the same assignment as
 * csc_kmeans_assign without best-distance sums or workspace: labels and best_d2 as there.
 * Its split centroids live in a static device array of the library (256 KiB per device,
 * held until the process ends), so it takes k <= 240 and d <= 256 (CSC_E_ARG beyond) and
 * calls no allocating routine.  Every call on a device uses that device's one array: calls
 * that overlap on one device race.  Asynchronous. */
csc_status csc_kmeans_assign_noalloc(const void* F, csc_dtype f_dt, int64_t ldf, int64_t n,
                                     int d, const float* C, int k, int32_t* labels,
                                     float* best_d2, void* stream);
csc_status csc_kmeans_update(const void* F, csc_dtype f_dt, int64_t ldf, int64_t n, int d,
                             const int32_t* labels, int k, float* C, int32_t* counts,
                             void* work, size_t work_bytes, void* stream);
csc_status csc_kmeans_seed(const void* F, csc_dtype f_dt, int64_t ldf, int64_t n, int d,
                           int k, const double* u, float* C, int32_t* idx, void* work,
                           size_t work_bytes, void* stream);
csc_status csc_kmeans(const void* F, csc_dtype f_dt, int64_t ldf, int64_t n, int d, int k,
                      int iters, int init, uint64_t seed, uint64_t stream_id, float* C,
                      int32_t* labels, double* objective, void* work, size_t work_bytes,
                      void* stream);

/* Compressive k-means (Sec. 2.2, Step 2): k-means on n_sample nodes drawn i.i.d. with
 * probability proportional to ||theta_i||^2 (a variable density; node i for a uniform u when
 * C_{i-1} <= u W < C_i over the prefix sums C of the squared row norms), then each cluster
 * indicator interpolated to every node by Tikhonov regularisation,
 *     x_j = argmin_x ||P^{-1/2} (M x - y_j)||^2 + gamma x^T L^r x
 * (M selects the sampled rows, P = diag(n_sample p_omega)), solved by preconditioned
 * conjugate gradients on the k columns (each product with L is one pass of the fused
 * recurrence) until every column's residual is below cg_tol times its right-hand side or
 * cg_iters iterations; node i gets argmax_j x_j[i] (ties to the lowest j).
 * F: device n x d features (F32 or BF16, ldf), n from the graph; k <= 256,
 * k <= n_sample <= n, 1 <= r <= 8, gamma > 0.  Random draws: uniforms of (seed,
 * sample_stream) for the samples and of (seed, kmeans_stream) for k-means++.  Outputs:
 * labels (device int32[n]); optionally the samples and their labels (device int32[n_sample])
 * and X (device float n x k); *cg_iters_done (host, nullable).  work:
 * csc_compressive_workspace_bytes(n, d, k, n_sample).  Synchronising. */
size_t csc_compressive_workspace_bytes(int64_t n, int d, int k, int n_sample);
csc_status csc_compressive_kmeans(csc_graph g, const void* F, csc_dtype f_dt, int64_t ldf, int d,
                                  int k, int n_sample, int r, double gamma, int lloyd_iters,
                                  int cg_iters, double cg_tol, uint64_t seed,
                                  uint64_t sample_stream, uint64_t kmeans_stream, int32_t* labels,
                                  int32_t* samples, int32_t* sample_labels, float* X,
                                  int* cg_iters_done, void* work, size_t work_bytes, void* stream);

/* ---------------------------------------------------------------------------------
 * Dynamic compressive spectral clustering (Algorithm 1, Sec. 4.1).
 *
 * The state keeps the n x d features Theta as a FIFO of columns, of which each snapshot
 * replaces the q d = round((1 - p) d) oldest (for p <= 1/2 the kept columns are exactly
 * those filtered on G_{t-1}), the cut-off of the previous snapshot, and the previous labels.
 *  - The first call runs static CSC on G_1 (Algorithm 1 steps 1-2): d signals, their
 *    moments, an n_cand-step dichotomy on [0, lmax], the filter at the found cut-off,
 *    k-means.
 *  - Each later call (steps 4-8): draws q d fresh signals, filters them on G_t with the
 *    previous filter, estimates their eigencount c = <R, h(L) R> / (sigma2 q d); when
 *    |c - k| > tau it computes their moments, bisects from the previous cut-off
 *    ([lambda, lmax] when c < k, [0, lambda] otherwise, lambda clipped to this snapshot's
 *    lmax) and filters them again; the
 *    result replaces the oldest block of Theta; k-means on Theta gives the labels.
 * Random draws: Philox streams 16 t + 1 (signals, variance 1/d) and 16 t + 2 (k-means++
 * uniforms), key `seed`.  feat_dt: storage of Theta and of the fresh signals (F32 or
 * BF16); iterates follow opts->iter_dt.  q d = round((1 - p) d) must lie in [1, d]; the
 * fresh block replaces the q d oldest columns, taken cyclically from a cursor that advances
 * by q d mod d, so any p works (a block that wraps past column d is staged and copied).
 * csc_dynamic_step writes labels (device int32[n]) and returns lambda_t, whether the
 * filter was refined and the eigencount of the fresh columns.  Synchronising.
 */
typedef struct {
  double lmax;        /* spectrum bound; 0 -> each graph's own (csc_lmax, iters 0) */
  double tau;         /* acceptance half-width, <= 0 -> max(0.5, 2 sqrt(2 k / (q d))) */
  int n_cand;         /* dichotomy steps, 0 -> 16 */
  int lloyd_iters;    /* Lloyd rounds after seeding, < 0 -> 20 */
  int init;           /* 0: k-means++ every snapshot; 1: warm start from previous labels */
  csc_dtype iter_dt;  /* storage of the recurrence iterates (F32, BF16, F16, BF16S, F16S) */
  int keep_iterates;  /* -1: keep all m + 1 iterates of the fresh block when they fit in free
                         device memory and m < 256 (a refinement then recombines them, in FP64,
                         instead of running the recurrence again); 0: never; 1: always
                         (CSC_E_NOMEM when they do not fit, CSC_E_ARG when m >= 256).  Where
                         two sets of kept iterates fit, csc_dynamic_steps runs the next
                         snapshot's (or batch's) recurrence beside the current one's
                         recombination, refinement and k-means */
  int batch;          /* csc_dynamic_steps: fresh blocks of up to `batch` (<= 8) snapshots are
                         filtered together, one launch per recurrence step: from kept
                         iterates, or, where they are not kept, as one-pass batches whose
                         snapshots are filtered again when their cut-off moves (0 or 1 -> one
                         snapshot at a time) */
  int use_graph;      /* non-zero: the recurrence launches are captured once in a HIP graph
                         and replayed for every snapshot (or batch) */
  int variant;        /* recurrence kernel shape (row group x column tile) for the fresh
                         block, e.g. the one csc_autotune picked on the first snapshot;
                         -1: the widest tile not wider than (1 - p) d */
  int track_similarity; /* non-zero: keep a device copy of the previous snapshot's operator
                         and report ||L_t - L_{t-1}||_F per snapshot (csc_dyn_similarity) */
  int sim_probes;     /* s in [0, (1 - p) d]: also estimate the spectral distance
                         ||H_k^t - H_k^{t-1}||_F as ||h(L_t) R_s - h(L_{t-1}) R_s||_F /
                         sqrt(s / d), with R_s the first s fresh signals and h the previous
                         filter on both graphs (one extra filter of s columns) */
  double refresh_budget; /* > 0 (needs sim_probes > 0): a snapshot where p times the estimate
                         exceeds the budget (the reuse term of Thm 4.1) is processed as static
                         CSC: all d columns drawn from its signal stream, a dichotomy on
                         [0, lmax], the ring restarted.  Any of the three similarity options
                         makes csc_dynamic_steps process snapshots one at a time. */
} csc_dyn_opts;

csc_status csc_dyn_create(int64_t n, int d, int k, double p, int m, csc_damping damp,
                          csc_dtype feat_dt, uint64_t seed, const csc_dyn_opts* opts,
                          csc_dyn* out);
csc_status csc_dynamic_step(csc_dyn st, csc_graph g_t, int32_t* labels, double* lambda_t,
                            int* refined, double* count, void* stream);
/* S snapshots in order (Algorithm 1 steps 4-8 for each): the fresh signals of up to
 * opts->batch snapshots are filtered in one batched recurrence (their graphs must share n
 * and the value type), then each snapshot's eigencount check, refinement, ring update and
 * k-means run in order, so the results equal S calls to csc_dynamic_step.  The state's own
 * non-blocking stream runs the recurrences and events order it against `stream`: with two
 * buffers of kept iterates the next batch's recurrence runs beside the current batch's
 * k-means, and with one buffer and batch 1 the next snapshot's recurrence starts once the
 * current snapshot's recombination and refinement are enqueued.  labels[i]: device int32[n]
 * per snapshot; lambdas, refined, counts: host arrays of S or NULL.  Synchronising; after
 * an error the state's stream is drained before the call returns. */
csc_status csc_dynamic_steps(csc_dyn st, const csc_graph* graphs, int S, int32_t* const* labels,
                             double* lambdas, int* refined, double* counts, void* stream);
/* Similarity record of snapshot t (1-based, already processed): the edge distance and the
 * spectral-distance estimate (-1 where not computed: t = 1 or the option off) and whether
 * the refresh rule fired.  Host call, no device work. */
csc_status csc_dyn_similarity(csc_dyn st, int t, double* rho_edge, double* rho_hat,
                              int* refreshed);
/* Checkpoint and resume of a dynamic state.  The state carried from one snapshot to the
 * next is Theta, the cut-off lambda_t, the ring cursor, the snapshot counter t, the
 * centroids and the labels (Algorithm 1 steps 4-8 read nothing else); the random draws are
 * functions of (seed, t), so a state imported into a fresh handle continues the sequence
 * bit for bit.  The host buffer holds a csc_dyn_header, then Theta (n x d row-major,
 * feat_dt), the centroids (float[k * d]) and the labels (int32[n]); its size is
 * csc_dyn_state_bytes.  A caller may edit the header's lambda (e.g. to force a refinement).
 * The copy of the previous operator kept for similarity tracking is not part of the state:
 * the first snapshot after an import reports no similarity.  Both calls synchronise `stream`;
 * export needs t >= 1 (CSC_E_STATE), import checks that n, d, k, m, q d, feat_dt and seed
 * match the handle's (CSC_E_ARG). */
typedef struct {
  uint64_t magic;   /* 0x31304e5944435343, "CSCDYN01" in little-endian bytes */
  int64_t n;
  int32_t d, k, m, qd;
  int32_t feat_dt, t, cursor, reserved;
  uint64_t seed;
  double lambda;
} csc_dyn_header;
size_t csc_dyn_state_bytes(csc_dyn st);
csc_status csc_dyn_export(csc_dyn st, void* host_buf, size_t bytes, void* stream);
csc_status csc_dyn_import(csc_dyn st, const void* host_buf, size_t bytes, void* stream);
/* Device view of Theta (n x d, type *dt, leading dimension *ld) and the centroids
 * (float[k * d]).  Valid until destroy. */
csc_status csc_dyn_features(csc_dyn st, const void** theta, csc_dtype* dt, int64_t* ld,
                            const float** centroids);
csc_status csc_dyn_destroy(csc_dyn st);

/* ---------------------------------------------------------------------------------
 * Adjoint of csc_cheb_filter (FP32).  Given G = dl/dY (device n x w, float, ldg), returns
 *   dX = sum_j a_j T_j(L~)^T G (device float n x w, lddx; NULL to skip),
 *   da[j] = <G, T_j(L~) X> (device double[m + 1] or NULL),
 *   dA[e] = dl/dA_e for every stored entry e of A (device float[nnz] or NULL), each entry
 *           a parameter of its own (the transposed product reads A's mirror entries);
 * by the reverse recurrence Zb_j = a_j G + 2 L~^T Zb_{j+1} - Zb_{j+2}, with the forward
 * iterates recomputed from checkpoints taken every ckpt_every steps (0 -> ceil(sqrt(m))).
 * X: device float n x w (ldx).  work: csc_cheb_backward_workspace_bytes(n, w, m,
 * ckpt_every).  Asynchronous.  Defined for the normalized Laplacian; a combinatorial
 * graph returns CSC_E_ARG.
 */
/* Chain of the adjoint from A's entries to the edge weights (Sec. 2.1: A = D^{-1/2} W
 * D^{-1/2} with d = W 1; normalized Laplacian only, CSC_E_ARG otherwise).  dA: device
 * float[nnz], dl/dA_e per stored entry as csc_cheb_filter_backward returns it.  dW: device
 * double[nnz], the derivative with respect to the symmetric weight of each entry's edge
 * (the same value on (i, j) and (j, i)): with s = D^{-1/2}, q_i = sum over the entries e of
 * row i of dA_e A_e + dA_m(e) A_m(e) (m(e) the mirror entry) and
 * g_ij = dA_ij s_i s_j - q_i s_i^2 / 2, dW_ij = g_ij + g_ji.  FP64 arithmetic on the stored
 * values of A (BF16 values carry their rounding into q).  work: device scratch of
 * csc_weight_grad_workspace_bytes(n) bytes.  Builds the mirror index on first use.
 * Asynchronous. */
size_t csc_weight_grad_workspace_bytes(int64_t n);
csc_status csc_weight_grad(csc_graph g, const float* dA, double* dW, void* work,
                           size_t work_bytes, void* stream);
size_t csc_cheb_backward_workspace_bytes(int64_t n, int w, int m, int ckpt_every);
csc_status csc_cheb_filter_backward(csc_graph g, double lmax, int m, const double* a,
                                    const float* X, int64_t ldx, const float* G, int64_t ldg,
                                    int w, float* dX, int64_t lddx, double* da, float* dA,
                                    int ckpt_every, void* work, size_t work_bytes,
                                    void* stream);

/* ---------------------------------------------------------------------------------
 * Measurement.  When enabled, csc_cheb_filter / csc_cheb_moments and the recurrences of the
 * dynamic calls record a pair of HIP events on their stream around their sequence of
 * recurrence-step kernels, and csc_timing_read sums, over the calls since the last reset,
 * the elapsed time, the number of step kernels and their algorithmic bytes (synchronising
 * on the recorded events).  The measurement state is one per process, not per thread or
 * device: enable, read and reset it from one thread while no other thread issues calls.
 */
csc_status csc_timing_enable(int on);
csc_status csc_timing_reset(void);
csc_status csc_timing_read(double* ms, int64_t* launches, double* bytes);

/* Random-gather probe (a measurement aid, not a step of the method): the ceiling of the
 * recurrence step's neighbour gathers on this memory system.  For the n_rows rows of a CSR
 * pattern (rowptr: device int32[n_rows + 1], colidx: device int32[nnz]) and a table of rows
 * of row_bytes bytes (64, 128, 256 or 512; device, 16-byte aligned), every row's group of
 * row_bytes / 16 lanes reads the table rows its column indices name, 16 bytes per lane and
 * eight loads in flight, as the step kernel does, and writes the XOR of what it read:
 * out[r * (row_bytes / 16) + q] (device uint32).  The caller guarantees that every column
 * index addresses a row of the table (nothing is checked on the device).  Asynchronous. */
csc_status csc_gather_probe(const int32_t* rowptr, const int32_t* colidx, int64_t n_rows,
                            const void* table, int row_bytes, uint32_t* out, void* stream);

/* Kernel-shape selection for the recurrence step of graph g at width w: candidate row
 * groups and column tiles are timed on the device and the fastest is kept in the handle
 * (variant index written to *variant).  Synchronising; uses `work` like csc_cheb_filter. */
csc_status csc_autotune(csc_graph g, int w, csc_dtype iter_dt, void* work, size_t work_bytes,
                        void* stream, int* variant);
/* Force a variant (-1 = heuristic default) for graph g and width class of iter_dt. */
csc_status csc_set_variant(csc_graph g, csc_dtype iter_dt, int variant);

#ifdef __cplusplus
}
#endif
#endif /* CSC_H */
