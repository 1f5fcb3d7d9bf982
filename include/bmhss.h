/*
 * bmhss -- MI355X (gfx950) library for the weakly singular Burton-Miller (WSBM)
 * Nystrom system of 2D TE-mode transmission scattering and its proxy-surface
 * HSS fast direct solver.
 *
 * Paper: "Proxy-surface-based fast direct solver for TE-mode scattering problems
 * on distributed memory systems" (Matsumoto, Yokota).
 *
 * Conventions used by every entry point
 * -------------------------------------
 *  - Complex numbers are interleaved FP64 (re, im), the layout of
 *    torch.complex128 / std::complex<double>.
 *  - Unknowns are node-interleaved: unknown 2j is u_j (the field), unknown 2j+1
 *    is q_j (the scaled normal derivative, Sec. II).  Row 2i holds the first
 *    row of Eq. (3) at node i, row 2i+1 the second row.
 *  - Matrices are row-major; `ld` is the leading dimension in complex elements.
 *  - Array arguments documented as "device" must be device pointers (HIP
 *    memory of the current device); "host" arguments are host pointers.  The
 *    caller owns every array; the library owns the opaque handles it creates
 *    and keeps its own device copy of the node data.
 *  - Device work is enqueued on the caller's stream and is asynchronous unless
 *    stated otherwise.  A handle must not be used from several host threads at
 *    once without external synchronisation.
 *  - Every call returns a status code.  On BM_EINVAL nothing has been enqueued.
 *    bm_last_error() returns a thread-local message for the last failure.
 */
#ifndef BMHSS_H
#define BMHSS_H

#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    BM_OK = 0,
    BM_EINVAL = 1,    /* bad shape, non-finite input, clockwise curve, k <= 0, ... */
    BM_ENOMEM = 2,    /* device or host allocation failed */
    BM_EHIP = 3,      /* HIP runtime error */
    BM_ESINGULAR = 4, /* zero pivot in an LU factorisation */
    BM_ESTATE = 5     /* handle in the wrong state */
};

typedef struct bm_geom bm_geom;
typedef struct bm_problem bm_problem;
typedef struct bm_hss bm_hss;

/* Material constants: wavenumbers k_j = omega sqrt(eps_j mu_j) and permittivities
 * of the exterior (0) and interior (1) media (Sec. II, Table I).  The
 * Burton-Miller constant is alpha = i/k0 (stated after Eq. (2)). */
typedef struct {
    double k0, k1, eps0, eps1;
} bm_media;

/* Message of the last failing call on this host thread ("" if none). */
const char* bm_last_error(void);

/* ---- Boundary discretisation (Sec. II; Nystrom method with trapezoidal nodes) ----
 * ncurves closed curves, curve c sampled at n_per_curve[c] >= 8 equispaced
 * parameter values t_j = 2 pi j / n_c, counter-clockwise.  xyd is a 6 x N_total
 * row-major FP64 array: rows x, y, x'(t), y'(t), x''(t), y''(t); curves are
 * concatenated.  xyd is a device pointer if on_device != 0, else a host pointer.
 * The library computes, on the device, outward normals n = (y', -x')/|x'|,
 * weights w = (2 pi/n_c)|x'| and curvature, and keeps them; it also keeps a
 * host copy of the node coordinates x, y (16 bytes per node), from which the
 * HSS build lays out its tree without reading the device back.  Validation
 * (finite values, non-degenerate speed, counter-clockwise orientation) is done
 * on the host; this call synchronises `stream`.  Returns BM_EINVAL on bad
 * input. */
int bm_geom_create(int ncurves, const int64_t* n_per_curve, const double* xyd, int on_device,
                   hipStream_t stream, bm_geom** out);
int bm_geom_destroy(bm_geom* g);
/* Total number of nodes, or -1 for a null handle. */
int64_t bm_geom_size(const bm_geom* g);
/* Copy the node data to `soa` (device, 6 x N row-major: x, y, nx, ny, w, kappa). */
int bm_geom_nodes(const bm_geom* g, double* soa, hipStream_t stream);

/* ---- Problem: geometry + media.  The geometry must outlive the problem. ---- */
int bm_problem_create(const bm_geom* g, const bm_media* media, bm_problem** out);
/* Several independent scatterers in one problem (the batched workload): the
 * curves are split into nbodies bodies, body_of_curve[c] (host) giving the
 * body of curve c; it must run 0, .., 0, 1, .., nbodies - 1 (consecutive curves,
 * every body at least one curve).  media[b] (host) are body b's media.  The
 * system is block diagonal: pairs in different bodies are zero blocks, every
 * body has its own incident field and far field, and the HSS build factors the
 * bodies as a forest (one tree per body, the levels of all trees batched).
 * bm_problem_create(g, media) is the one-body case. */
int bm_problem_create_bodies(const bm_geom* g, int nbodies, const int32_t* body_of_curve,
                             const bm_media* media, bm_problem** out);
int bm_problem_destroy(bm_problem* p);

/* ---- Right-hand side of Eq. (3) for a plane wave (Sec. IV) ----
 * u_in = exp(i k0 (cos angle, sin angle) . x); rhs (device, 2N complex):
 * rhs[2i] = 0, rhs[2i+1] = -u_in(x_i) - alpha du_in/dn(x_i). */
int bm_rhs_plane_wave(const bm_problem* p, double angle, double* rhs, hipStream_t stream);

/* ---- Right-hand side of Eq. (3) for any incident field ----
 * uin, dn_uin (device, N complex): the incident field u_in and its outward
 * normal derivative du_in/dn at the nodes, e.g. of a point source or of a sum
 * of plane waves; rhs (device, 2N complex): rhs[2i] = 0,
 * rhs[2i+1] = -u_in(x_i) - alpha du_in/dn(x_i), alpha = i/k0 of node i's body.
 * rhs must not alias uin or dn_uin.  Asynchronous on `stream`. */
int bm_rhs_incident(const bm_problem* p, const double* uin, const double* dn_uin, double* rhs,
                    hipStream_t stream);

/* ---- Matrix entries: Eq. (3) / Eq. (5), one-point corrected diagonal ----
 * Full matrix (device, 2N x 2N complex, row-major, ld >= 2N). */
int bm_assemble_dense(const bm_problem* p, double* A, int64_t ld, hipStream_t stream);

/* Block A(rows, cols) for node index lists (device int64 arrays, values in
 * [0, N)); out (device) is 2nr x 2nc complex with leading dimension ld >= 2nc.
 * Pairs with rows[a] == cols[b] get the corrected diagonal block of Eq. (5)
 * (delta_ij = 1); pairs in two different bodies are zero blocks.  Indices are
 * not validated on the device: out-of-range values are the caller's error.
 * prec = 0: FP64 arithmetic; prec = 1: FP32 arithmetic (coordinate
 * differences and the phase reduction of large arguments in FP64), entries
 * rounded to FP32 accuracy and stored as FP64 complex -- for blocks that only
 * select skeletons.  The entries come from the same generator the HSS build
 * runs; a small device buffer (slot lists) is allocated and released on
 * `stream`.  nr, nc < 2^30. */
int bm_assemble_block(const bm_problem* p, const int64_t* rows, int64_t nr, const int64_t* cols,
                      int64_t nc, double* out, int64_t ld, int prec, hipStream_t stream);

/* Proxy blocks for the proxy-surface compression (Sec. I and III; the proxy
 * method of Martinsson-Rokhlin).  Proxy points are pseudo-nodes given by pts
 * (device, 5 x P row-major: x, y, nx, ny, w).  The same pair formula is used
 * with no diagonal term.  dir = 0: node targets x proxy sources, out is
 * 2n x 2P (ld >= 2P); dir = 1: proxy targets x node sources, out is 2P x 2n
 * (ld >= 2n).  nodes: device int64 list of node indices.  Proxy points must
 * not coincide with nodes.  A proxy point takes the media of the node it is
 * paired with, and the interior (k1) terms are kept.  prec as in
 * bm_assemble_block.  The generator's point table (the N nodes and the P
 * proxy points) is copied into a device buffer allocated and released on
 * `stream`. */
int bm_assemble_proxy(const bm_problem* p, const int64_t* nodes, int64_t n, const double* pts,
                      int64_t P, int dir, double* out, int64_t ld, int prec, hipStream_t stream);

/* y = A x without storing A (device, 2N complex each): the matrix entries are
 * generated on the fly and reduced. */
int bm_matvec(const bm_problem* p, const double* x, double* y, hipStream_t stream);

/* bm_matvec for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and the same result, bit for bit, but the block partial sums go
 * to a fixed buffer of 16 MiB (2^21 doubles) that the library holds in device
 * memory on every GPU it runs on until the process ends, instead of a buffer
 * it allocates.  The buffer needs 4 N ceil(B / 2048) doubles, B the largest
 * body in nodes (one body: N <= 32768); larger problems get BM_EINVAL
 * (use bm_matvec).  Nothing is allocated and nothing needs clearing (every
 * partial sum is written before it is read).  All calls on one GPU share the
 * buffer: calls that overlap on one GPU (different streams, no ordering)
 * race and give wrong results; calls ordered on one stream are safe.
 * x, y: device, 2N complex, must not alias.  Asynchronous on `stream`. */
int bm_matvec_noalloc(const bm_problem* p, const double* x, double* y, hipStream_t stream);

/* Far field of the scattered field from a solution phi = (u_0, q_0, u_1, ...)
 * (device, 2N complex), at nang observation angles (device FP64); uinf (device,
 * nbodies * nang complex, body b's far field at uinf[b * nang + a], each body
 * about the origin with its own k0).  u_sc(x) ~ exp(i k0 |x|)/sqrt(|x|)
 * uinf(x/|x|), from the exterior representation u_sc = D_k0[u] - S_k0[eps0 q]
 * (remark after Eq. (3)). */
int bm_far_field(const bm_problem* p, const double* phi, const double* angles, int64_t nang,
                 double* uinf, hipStream_t stream);

/* ---- Proxy-surface HSS direct solver (Sec. III) ----
 * The boundary nodes are split by a perfect binary tree of contiguous index
 * ranges (Fig. 2) down to leaves of about `leaf` nodes.  At every level each
 * box is compressed by an interpolative decomposition (ID) of its interactions
 * with the near boxes (other boxes' active unknowns inside its proxy circle)
 * and with `proxy_points` pseudo-nodes on a circle of radius
 * proxy_ratio * (box radius).  The ID is column-pivoted QR with relative
 * tolerance id_tol, of the stacked matrix or of a random sketch of it (opts
 * sketch); skeletons are sets of unknowns shared by rows and columns.
 * The factorisation is the Martinsson-Rokhlin recursion: per box
 * Dhat = (T^T D^-1 T)^-1, E = D^-1 T Dhat, F^T = Dhat T^T D^-1,
 * G = D^-1 - D^-1 T Dhat T^T D^-1, and the inverse of the dense root
 * system.  Inverses pivot rows inside diagonal blocks of at most 64 only:
 * Gauss-Jordan elimination up to that size, above it a 2 x 2 Schur-complement
 * recursion, except for the single root of a one-body problem of at most 4096
 * unknowns, which is inverted by block Gauss-Jordan over 64-column panels. */
typedef struct {
    int64_t leaf;          /* target leaf size in nodes (>= 4) */
    double proxy_ratio;    /* proxy circle radius / box radius (> 1) */
    int64_t proxy_points;  /* points per proxy circle (>= 8) */
    double id_tol;         /* relative ID tolerance (0 < tol < 1) */
    int64_t sketch;        /* 0: CPQR of each box's stacked near/proxy matrix;
                              p > 0: CPQR of a Gaussian sketch of it with
                              min(rows, unknowns + p) rows (randomized ID);
                              -1: the library's tuned value */
    int64_t proxy_adapt;   /* 0: proxy_points on every proxy circle; 1: per box
                              max(proxy_points, ceil(2 k R_p) + 32), k the larger
                              wavenumber of the box's body, R_p the proxy radius */
    double max_rank_ratio; /* 0: compress every body up to its top level or until a
                              box has no far unknowns; r in (0, 1]: also stop a body
                              (its current boxes' skeletons become its dense root)
                              once a level's skeletons keep more than r of its
                              unknowns -- at high frequency the ranks grow with the
                              box size and compressing further does not pay;
                              -1: the library's tuned value */
    int64_t kernel_timing; /* 1: time every launch of the batched GEMM and Gauss-Jordan
                              kernels with HIP events (bm_hss_stats_t gemm_* and
                              inv_*; adds an event pair per launch); 0: off */
    int64_t proxy_fp32;    /* 1: node x proxy blocks in FP32 arithmetic (they only
                              select skeletons; near, skeleton and diagonal blocks,
                              the ID and the factors stay FP64); 0: FP64 */
} bm_hss_opts;

typedef struct {
    int32_t levels;            /* tree depth: the leaves are level `levels` */
    int32_t compressed_levels; /* levels compressed by the proxy ID */
    int32_t root_size;         /* unknowns of the dense root system */
    int32_t guard_stops;       /* bodies whose compression the ID work guard ended:
                                  a box's stacked ID matrix above 2^26 entries, or a
                                  body's above 2^31 at one level (its skeletons then
                                  form its dense root) */
    int64_t max_rank;          /* largest skeleton (unknowns) over all boxes */
    int64_t entries;           /* matrix entries generated during the build */
    int64_t pairs;             /* node pairs evaluated (each gives a 2x2 block) */
    double seconds_generate;   /* time in entry-generation kernels (HIP events) */
    double seconds_compress;   /* time in the ID kernels (HIP events) */
    double seconds_factor;     /* time in inversion and GEMM kernels (HIP events) */
    double seconds_total;      /* wall time of bm_hss_build */
    /* the step-wise CPQR (the ID): launches of its step kernel, the bytes each
     * executed step must move at least (the trailing columns read and written
     * once, the Householder column and the column norms), and the time from
     * the first to the last step launch of every level (HIP events on the
     * build stream, so launch gaps are included) */
    int64_t cpqr_launches;
    double cpqr_bytes;
    double seconds_cpqr;
    /* the sketch and max_rank_ratio the build used (tuned values resolved) */
    int64_t sketch;
    double max_rank_ratio;
    /* levels whose boxes fit one workgroup (at most 128 unknowns and 160 ID
     * rows) run the whole CPQR in one launch instead of the step kernels:
     * those launches, their algorithmic bytes (each matrix read and written
     * once, pivots and diagonal written) and their event-timed duration; the
     * three step-wise figures above exclude them */
    int64_t cpqr_fused_launches;
    double cpqr_fused_bytes;
    double seconds_cpqr_fused;
    /* with opts.kernel_timing: launches of the batched GEMM kernel (rocBLAS
     * calls excluded), their algorithmic flops (8 M N K per complex product)
     * and summed event-timed durations; the same for the batched Gauss-Jordan
     * kernels (8 n^3 flops per inverted block); zero otherwise */
    int64_t gemm_launches;
    double gemm_flops;
    double seconds_gemm;
    int64_t inv_launches;
    double inv_flops;
    double seconds_inv;
    /* with opts.kernel_timing: the sketch launches (their algorithmic flops,
     * 4 l m n for an l-row sketch of an m x n complex matrix, and summed
     * durations) and the FP64 entry-generation launches (pairs evaluated and
     * summed durations); zero otherwise */
    int64_t sketch_launches;
    double sketch_flops;
    double seconds_sketch;
    int64_t gen_launches;
    double gen_pairs;
    double seconds_gen;
} bm_hss_stats_t;

/* Build the factorisation; synchronises `stream` once per level to read the
 * ranks back, and returns after the whole build has completed on the stream. */
int bm_hss_build(const bm_problem* p, const bm_hss_opts* opts, hipStream_t stream, bm_hss** out);
/* x = A^{-1} b for nrhs right-hand sides (device, 2N x nrhs complex, each
 * right-hand side contiguous: b[r*2N + i]).  x may alias b.  The solve is an
 * upward sweep F^T b, a dense product with the inverted root system and a
 * downward sweep G b + E x.  Returns after the solve has completed on the
 * stream. */
int bm_hss_solve(const bm_hss* h, const double* b, double* x, int64_t nrhs, hipStream_t stream);
/* x = A^{-T} b (plain transpose, no conjugation; same layout as bm_hss_solve),
 * from the same factors: the solve's data flow reversed with every factor
 * transposed (y_0 = b, G^T and E^T per box from the leaves up, the transposed
 * root inverse, then (F^T)^T per box from the root down).  This is the adjoint
 * solve A^T lam = g of a shape derivative.  x may alias b.  Returns after the
 * solve has completed on the stream. */
int bm_hss_solve_transpose(const bm_hss* h, const double* b, double* x, int64_t nrhs, hipStream_t stream);
/* The same solve (transpose = 0) or transposed solve (transpose = 1) replayed
 * from a HIP graph: the first call for a given (nrhs, transpose) records the
 * solve's level sweeps once -- job descriptors uploaded to device memory, the
 * launches captured on a library stream -- and every call then copies b into
 * the graph's input buffer, launches the graph on `stream` and copies the
 * result to x.  Unlike bm_hss_solve it does not synchronise: it returns as soon
 * as the work is enqueued.  Calls with the same (nrhs, transpose) share one
 * input/output buffer pair, so they must be ordered on one stream (or
 * synchronised); bm_hss_destroy waits for the last launch of every graph.  The
 * graph holds device memory (the sweep buffers, 2N x nrhs in and out) until
 * bm_hss_destroy.  Every product of the graph runs in the library's own
 * batched GEMM kernel (library GEMM calls are not captured), so for a very
 * large root the eager solve, which hands large products to rocBLAS, can be
 * faster.  bm_hss_build records the (nrhs = 1, transpose = 0) graph itself,
 * on the host while the GPU inverts the dense root, so that the first such
 * call only replays it. */
int bm_hss_solve_graph(const bm_hss* h, const double* b, double* x, int64_t nrhs, int transpose,
                       hipStream_t stream);
int bm_hss_stats(const bm_hss* h, bm_hss_stats_t* out);

/* In-place inverse of one dense complex n x n matrix on the device, by the
 * method the HSS factorisation uses for its diagonal blocks and its dense root
 * (the inverses in the Martinsson-Rokhlin factors of the direct solver, paper
 * Sec. III): Gauss-Jordan with partial row pivoting for n <= 64; above that
 * block Gauss-Jordan over 64-column panels (n <= 4096), or the 2 x 2
 * Schur-complement recursion, rows pivoted within the 64 x 64 diagonal blocks.
 * a: device, interleaved complex128, element (i, j) at a[2 (i ld + j)],
 * overwritten by the inverse; 1 <= n <= 16384, n <= ld.  Returns after the
 * inverse has completed on the stream.  BM_ESINGULAR if a pivot is zero, not
 * finite or below 64 eps times the largest magnitude in its 64 x 64 diagonal
 * block (the kernels end normally; for n <= 64 the matrix is then left as it
 * was, above that its contents are unspecified).  Test hook: with
 * BMHSS_TEST_SINGULAR_ROOT=1 in the environment, bm_hss_build zeroes the first
 * row of its dense root before inverting it (and so returns BM_ESINGULAR). */
int bm_dense_inverse(double* a, int64_t n, int64_t ld, hipStream_t stream);

/* The sketch of the randomized interpolative decomposition (the ID of a box
 * then runs on Y instead of on its stacked near-field and proxy matrix, paper
 * Sec. III): Y = Omega X for a real l x m matrix Omega (row-major, leading
 * dimension ldo >= m) and a complex m x n matrix X (column j at x + 2 j m,
 * interleaved complex128), giving the complex l x n matrix Y (column j at
 * y + 2 j l).  All device pointers; the product runs on the FP64 matrix
 * cores, with the K range split over several workgroups (and the partial
 * products summed in a fixed order) when the tiles alone would leave most
 * compute units idle.  Returns after Y has been written.  EINVAL for sizes
 * out of range. */
int bm_sketch(const double* omega, int64_t ldo, const double* x, int64_t m, int64_t n, int64_t l, double* y,
              hipStream_t stream);

/* The interpolative decomposition that picks each box's skeleton (the ID of
 * the proxy-surface compression, paper Sec. III; skeleton indices as in
 * Martinsson and Rokhlin), for a batch of nb complex matrices at once: the
 * kernels of bm_hss_build's ID step, on caller-given matrices.  Matrix b is
 * m[b] x n[b] (host arrays), stored by columns (column j at x + 2 (o_b + j m[b]),
 * interleaved complex128, device, o_b = sum over a < b of m[a] n[a]); it is
 * factored by Householder QR with column pivoting (at step k the remaining
 * column of largest 2-norm over rows k.., lowest index on ties) until
 * |R_kk| <= tol |R_00| or min(m, n) steps; the number of steps taken is the
 * rank k_b, written to ranks[b] (host).  x is overwritten by the factorisation.
 * perm + p_b (device, n[b] entries, p_b = sum over a < b of n[a]) receives the
 * pivot order: the skeleton columns perm[0..k_b), then the other columns in
 * increasing order.  T + 2 t_b (device, room for n[b]^2 complex values,
 * t_b = sum over a < b of n[a]^2) receives the n[b] x k_b interpolation
 * matrix, row-major with row stride k_b: row perm[i] is e_i for i < k_b and
 * row perm[k_b + c] is column c of R11^-1 R12, so that column j of the matrix
 * is approximated by sum_i X[:, perm[i]] T[j][i]; the rest of each slot is
 * zeroed.  One workgroup factors a whole matrix when n <= 160 and m <= 160,
 * otherwise one launch per elimination step.  Returns after every output has
 * been written.  EINVAL: a null pointer, nb outside 1..65535, a size outside
 * 1..4096, tol outside [0, 1). */
int bm_interp_decomp(int32_t nb, const int32_t* m, const int32_t* n, double* x, double tol, int32_t* ranks,
                     int32_t* perm, double* T, hipStream_t stream);

/* Per compressed level (0 = leaves, up to compressed_levels - 1): sizes of the
 * ID problems and the ranks found.  EINVAL for a level out of range. */
typedef struct {
    int32_t boxes;          /* boxes on the level */
    int32_t max_unknowns;   /* largest box: active unknowns (columns of the ID) */
    int32_t max_rows;       /* largest stacked matrix: near + proxy rows per box */
    int32_t id_rows;        /* rows the CPQR ran on (max over boxes): the sketch
                               height, or max_rows without a sketch */
    int32_t min_rank;       /* smallest and largest skeleton, in unknowns */
    int32_t max_rank;
} bm_hss_level_t;
int bm_hss_level(const bm_hss* h, int level, bm_hss_level_t* out);

/* Releases the factors (to the library's device-memory cache, where the next
 * build can reuse them on any stream).  Waits for the graph-replayed solves;
 * every other call on h returns after its device work has completed. */
int bm_hss_destroy(bm_hss* h);
/* ---- Shape derivatives of far-field objectives (adjoint method) ----
 * The paper solves Eq. (3) for a fixed boundary; these entry points
 * differentiate the discrete solution with respect to the boundary samples.
 *
 * Far-field weights: g (device, 2N complex) such that body b's far field at
 * `angle` is u_inf,b = sum over b's unknowns k of g_k phi_k (the formula of
 * bm_far_field written per unknown). */
int bm_far_field_weights(const bm_problem* p, double angle, double* g, hipStream_t stream);

/* Derivative of L_b = g_b^T phi + lam^T (rhs - A phi) over each body b, with
 * phi and lam fixed, with respect to the six samples (x, y, x', y', x'', y'')
 * of every node, through the positions, normals, weights and curvatures the
 * geometry derives from them (Sec. II) and the one-point corrected diagonal:
 *   grad[q*N + i] = Re(coef_b dL_b / d s_q(i))   (device, 6 x N FP64 output),
 * g = far-field weights at obs_angle, rhs = the plane wave at inc_angle
 * (bm_rhs_plane_wave).  For phi = A^-1 rhs and A^T lam = g, dL_b is the
 * derivative of u_inf,b(obs_angle); coef (device, nbodies complex) weights
 * the bodies, e.g. coef_b = 2 conj(u_inf,b) for |u_inf,b|^2.  coef = NULL
 * takes that weight: grad is then the gradient of sum_b |u_inf,b(obs_angle)|^2.
 * phi, lam: device, 2N complex.  The pair sums use FP64 atomic additions, so
 * the last bits may differ between runs.  Asynchronous on `stream`. */
int bm_shape_derivative(const bm_problem* p, const double* phi, const double* lam, double inc_angle,
                        double obs_angle, const double* coef, double* grad, hipStream_t stream);

/* Samples of the closed curve x(t) = (cx, cy) + radius r(t) (cos t, sin t),
 * r(t) = 1 + sum_{j=1..M} (a_j cos jt + b_j sin jt), at t_i = 2 pi i / n:
 * xyd (device, 6 x n, the layout bm_geom_create takes); coef (device, 2M FP64)
 * = a_1..a_M, b_1..b_M.  The curve must stay star-shaped (r > 0) for the
 * geometry to be valid; that is checked by bm_geom_create. */
int bm_fourier_curve(const double* coef, int nmodes, double radius, double cx, double cy, int64_t n,
                     double* xyd, hipStream_t stream);
/* The chain rule of bm_fourier_curve: out[m] = sum over i and rows q of
 * grad[q*n + i] d xyd[q*n + i] / d coef_m (device, 2M FP64), e.g. a shape
 * derivative from bm_shape_derivative turned into d/d(a_1..a_M, b_1..b_M). */
int bm_fourier_chain(const double* grad, int64_t n, int nmodes, double radius, double* out, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* BMHSS_H */
