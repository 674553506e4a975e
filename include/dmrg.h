/*
 * dmrg.h -- C ABI of the MI355X two-site DMRG middle-site library
 * (libdmrg_hip.so).
 *
 * The calls follow the paper's statement of one two-site DMRG sweep
 * iteration (Zhai & Chan, "Low communication high performance ab initio
 * density matrix renormalization group algorithms", Appendix A and B):
 *
 *   integrals           -> ab initio Hamiltonian (Appendix B, first equation),
 *                          optionally one sub-Hamiltonian of the sum of
 *                          sub-Hamiltonians (Section II.B)
 *   dmrg_build_block    -> blocking (Appendix A, blocking formula) followed by
 *                          transformation (Appendix A, operator transformation)
 *                          site by site from an edge to the middle
 *   dmrg_normal_to_complementary
 *                       -> normal -> complementary transform of the mixed
 *                          NC/CN partition (Section III.A)
 *   dmrg_heff_create    -> blocking at the two dots and the list of sector
 *                          products of H_eff (Section II.D/II.E, "list of GEMMs
 *                          generated once for each site", Section II.G)
 *   dmrg_heff_apply     -> H_eff psi (Appendix A, effective eigenproblem)
 *   dmrg_davidson       -> Davidson solution of the effective eigenproblem
 *                          (also one iteration at a time: dmrg_davidson_step)
 *   dmrg_decimate       -> decimation: the new renormalized basis from the
 *                          reduced density matrix of the solution (Appendix A)
 *   dmrg_heff_renormalize, dmrg_renormalize
 *                       -> transformation of blocked operators into a new
 *                          renormalized basis (Appendix A)
 *   dmrg_query_workspace-> arena bytes of each call, host only
 *
 * Conventions shared with every caller:
 *   spin-orbital p = 2*i + s (s = 0 alpha, 1 beta), spatial i = 0..K-1;
 *   sector label (n_alpha, n_beta); site basis |0>,|a>,|b>,|ab>;
 *   left block Lb = sites [0, KL), dots d1 = KL, d2 = KL+1, right block
 *   Rb = [KL+2, K) (the middle step: KL = K/2 - 1; a sweep moves KL from 1
 *   to K-3 and back);
 *   a block grown by one site orders the rows of each enlarged sector by site
 *   state (0, a, b, ab), each segment holding the old block's sector
 *   q - q_site in the old block's order (sectors sorted by (n_alpha, n_beta));
 *   wavefunction: sub-blocks (a, s1, s2, b), ordered by Lb sector a, then s1,
 *   then s2 (b is fixed by the target); each m_a x m_b row-major.  n_vec
 *   vectors are stored one after another (stride = dmrg_heff_dim).
 *
 * Memory: the library never allocates device memory.  The caller hands one
 * device arena to dmrg_create; every operator, work list and Davidson vector
 * is carved out of it.  Calls fail with DMRG_E_WORKSPACE when it is too small.
 * Device pointers passed in (isometries, psi, sigma) stay owned by the caller.
 *
 * Errors: every call returns a dmrg_status; no exception or abort crosses the
 * ABI.  Arguments are checked before any device work.  HIP errors map to
 * DMRG_E_HIP with hipGetErrorString in dmrg_last_error().  Work is queued on
 * the caller's stream (a hipStream_t passed as void*); asynchronous faults
 * surface at the next synchronising call.  A context is not thread-safe.
 */
#ifndef DMRG_H
#define DMRG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t dmrg_status;
enum {
    DMRG_OK = 0,
    DMRG_E_ARG = -1,          /* invalid argument or shape */
    DMRG_E_SYMMETRY = -2,     /* integrals break t_ij = t_ji or 8-fold v symmetry */
    DMRG_E_WORKSPACE = -3,    /* arena too small */
    DMRG_E_HIP = -4,          /* HIP runtime error */
    DMRG_E_NONFINITE = -5,    /* NaN/Inf met in a Davidson vector */
    DMRG_E_STATE = -6,        /* call out of order (e.g. no integrals) */
    DMRG_E_UNSUPPORTED = -7   /* a size the kernels cannot address (an operand of 2^32 bytes or more) */
};

enum { DMRG_LEFT = 0, DMRG_RIGHT = 1 };
/* right-block schemes (left blocks are always NC: normal operators) */
enum { DMRG_SCHEME_NC = 0,   /* complementary operators (P, Q, R) on the right */
       DMRG_SCHEME_CN = 1 }; /* normal operators on the right, transformed at the middle */
enum { DMRG_F64 = 0, DMRG_F32 = 1 };
enum { DMRG_PREC_F64 = 0, DMRG_PREC_F32 = 1 };

typedef struct dmrg_ctx dmrg_ctx;
typedef struct dmrg_opset dmrg_opset;
typedef struct dmrg_heff dmrg_heff;

/* Block-sparse matrix with quantum-number-labelled sectors (a site
 * isometry A[k] of the MPS, Appendix A).  Block b maps enlarged sector
 * qn_row[2b..2b+1] (rows, enlarged basis order) to new sector
 * qn_col[2b..2b+1]; for an isometry qn_row == qn_col.  Data is row-major
 * rows[b] x cols[b] at element offset offset[b] of `data` (device, f64).
 * The metadata arrays are host arrays, copied by the library. */
typedef struct {
    int32_t n_blocks;
    const int32_t* qn_row;
    const int32_t* qn_col;
    const int64_t* rows;
    const int64_t* cols;
    const int64_t* offset;
    int32_t dtype;
    const void* data;
} dmrg_bsm;

typedef struct {
    int32_t max_iter;         /* cap on iterations (matvec rounds) */
    int32_t max_subspace;     /* vectors kept before a restart (>= 2*n_roots) */
    double tol;               /* converged when every residual norm <= tol */
    int32_t precision;        /* DMRG_PREC_F64, or DMRG_PREC_F32 for the mixed policy */
    double switch_tol;        /* mixed policy: FP32 matvecs while max residual > switch_tol */
    int32_t fixed_iters;      /* > 0: run exactly this many iterations (timing mode) */
    double precond_clamp;     /* diagonal preconditioner t = r / (theta - d) with |theta - d|
                                 clamped >= precond_clamp; 0 selects 0.1; < 0 disables the
                                 preconditioner (t = r) */
} dmrg_dav_opts;

typedef struct {
    int32_t iters;            /* iterations done */
    int32_t matvecs;          /* H_eff psi products (vector count) */
    int32_t matvecs_f32;      /* of which in FP32 */
    int32_t converged;        /* 1 if every residual <= tol */
    double max_residual;      /* final max residual norm */
    double ms_total;          /* wall time of the call (device events) */
    double ms_matvec;         /* time inside H_eff psi */
} dmrg_dav_stats;

const char* dmrg_status_string(dmrg_status s);
/* thread-local detail of the last error */
const char* dmrg_last_error(void);

/* Context on HIP device `device` with the caller's device arena. */
dmrg_status dmrg_create(dmrg_ctx** out, int32_t device, void* arena, int64_t arena_bytes);
void dmrg_destroy(dmrg_ctx* ctx);
/* bytes of the arena in use now / at peak */
int64_t dmrg_arena_used(const dmrg_ctx* ctx);
int64_t dmrg_arena_peak(const dmrg_ctx* ctx);

/* Integrals of the ab initio Hamiltonian (Appendix B): h1e[K*K] and
 * g2e[K^4] in chemists' order (ij|kl), host arrays (copied), e_core added to
 * H_eff.  With n_proc > 1 the context keeps only sub-Hamiltonian proc_id
 * (1-based) of the sum of sub-Hamiltonians (Section II.B, processor
 * assignment with the NC rule): t_ij scaled by [proc(p,i)+proc(p,j)]/2 and
 * v_ijkl kept when proc(p, sorted i,j,k,l) = 1.  Fails with DMRG_E_SYMMETRY
 * if h is not symmetric or g not 8-fold symmetric to 1e-12. */
dmrg_status dmrg_set_integrals(dmrg_ctx* ctx, int32_t K, int32_t n_elec, int32_t two_sz,
                               const double* h1e, const double* g2e, double e_core,
                               int32_t n_proc, int32_t proc_id);

/* Edge-to-middle build: blocking then transformation for n_sites sites from
 * the `side` edge (left: sites 0..n_sites-1; right: K-1 down to K-n_sites).
 * isometries[j] is the isometry adding the j-th site counted from that edge.
 * Left blocks hold normal operators; right blocks hold normal operators
 * (DMRG_SCHEME_CN) or complementary ones (DMRG_SCHEME_NC).  The operator set
 * lives in the context arena; free it with dmrg_opset_free. */
dmrg_status dmrg_build_block(dmrg_ctx* ctx, int32_t side, int32_t n_sites,
                             const dmrg_bsm* isometries, int32_t scheme,
                             dmrg_opset** out, void* stream);

/* Mixed NC/CN middle transform (Section III.A): replaces the two-index normal
 * operators of a CN right block by the complementary P, Q of every pair of
 * spin-orbitals to its left.  In place; cost O(K^4 M^2). */
dmrg_status dmrg_normal_to_complementary(dmrg_ctx* ctx, dmrg_opset* right, void* stream);

/* Layout of the two-site wavefunction in a caller's vector: one entry per
 * sub-block (a, s1, s2, b) -- left-block sector a = qn_left[2i..2i+1], dot
 * states s1 = site1[i], s2 = site2[i] (0..3 = |0>,|a>,|b>,|ab>); the right
 * sector b completes the target and the sub-block is m_a x m_b row-major at
 * element offset[i].  Every valid (a, s1, s2) must appear exactly once and
 * the sub-blocks must tile [0, dim) without gaps or overlaps (dim = the sum
 * of m_a m_b).  Host arrays, copied by the library. */
typedef struct {
    int32_t n_blocks;
    const int32_t* qn_left;
    const int32_t* site1;
    const int32_t* site2;
    const int64_t* offset;
} dmrg_psi_layout;

/* Blocking of the dots d1 (onto the left block) and d2 (onto the right
 * block, which must hold complementary operators) and the work list of
 * H_eff = sum over NC terms X^{L'} (x) Y^{R'} (Appendix A, effective
 * eigenproblem; Section II.G: the list of GEMMs is generated once for each
 * site and reused by every product).
 *   layout:    wavefunction layout of psi / sigma, or NULL for the default
 *              order (Lb sector a, then s1, then s2; contiguous);
 *   n_roots:   the largest vector batch one product serves at once (the
 *              partial-tile buffer is sized for it);
 *   precision: DMRG_PREC_F64 -- FP64 products only; DMRG_PREC_F32 -- FP32
 *              products as well (the FP32-mixed policy): the operators are
 *              rounded to binary32 copies here, once;
 *   flags:     DMRG_HEFF_GRAPH -- every product (dmrg_heff_apply, and so
 *              Davidson) replays a graph of its kernel launches, instantiated
 *              once per precision and vector batch, with the nodes' vector
 *              arguments updated per call;  DMRG_HEFF_AUTOTUNE (needs
 *              DMRG_PREC_F32) -- the work list's parameters (the number of
 *              equal-cost chunks heavy tiles are cut into, and the height
 *              from which tiles run on the tall kernel) are chosen by timing
 *              one FP32 product of each candidate (on n_roots vectors at
 *              once, the batch Davidson's products run on), then cached for
 *              the shape
 *              (the file named by DMRG_TUNE_CACHE, if set, keeps the cache
 *              across processes).  dmrg_heff_get_info reports the choice.
 *              Without it the list takes the defaults, or DMRG_BALANCE and
 *              DMRG_TALL_MIN from the environment.
 * DMRG_E_ARG for a layout that does not match the blocks; DMRG_E_WORKSPACE if
 * the arena cannot hold the blocked operators, lists and copies. */
enum { DMRG_HEFF_GRAPH = 1,      /* products replay a graph of their kernel launches */
       DMRG_HEFF_AUTOTUNE = 2 };  /* time candidate work lists at creation, keep the fastest */
dmrg_status dmrg_heff_create(dmrg_ctx* ctx, const dmrg_opset* left, const dmrg_opset* right,
                             const dmrg_psi_layout* layout, int32_t n_roots, int32_t precision,
                             int32_t flags, dmrg_heff** out, void* stream);
int64_t dmrg_heff_dim(const dmrg_heff* H);
typedef struct {
    int32_t flags;                /* as created */
    int32_t balance_target;       /* equal-cost chunks the work is cut into */
    int32_t tall_min_rows;        /* tiles of this many rows or more run on the tall kernel */
    int32_t tuned;                /* 0 defaults, 1 timed at creation, 2 from the cache */
    int32_t n_candidates;         /* candidates timed (tuned == 1), at most 8 */
    float candidate_ms[8];        /* FP32 product time of each */
    int32_t candidate_balance[8];
    int32_t candidate_tall_min[8];
    int32_t graphs;               /* product graphs instantiated */
    int64_t graph_launches;       /* products run as graph replays */
    int64_t tasks;                /* output tiles of the work list */
    int32_t reductions;           /* split tiles summed by the reduction */
    int64_t partial_elems;        /* elements of their partial tiles, per vector */
} dmrg_heff_info;
dmrg_status dmrg_heff_get_info(const dmrg_heff* H, dmrg_heff_info* info);
/* Readback of the layout in use (host arrays of capacity >= n, any may be
 * NULL): qn_left / qn_right [2 n], site1 / site2 [n], rows / cols / offset
 * [n].  Returns the number of sub-blocks. */
int32_t dmrg_heff_psi_layout(const dmrg_heff* H, int32_t n, int32_t* qn_left, int32_t* site1, int32_t* site2,
                             int32_t* qn_right, int64_t* rows, int64_t* cols, int64_t* offset);

/* sigma = H_eff psi for n_vec vectors (overwrite).  precision DMRG_PREC_F64:
 * psi, sigma are double; DMRG_PREC_F32: float (operators rounded to binary32
 * once, FP32 products with FP32 accumulation; DMRG_E_STATE if H was created
 * for FP64 only).  Vectors run in batches of n_roots. */
dmrg_status dmrg_heff_apply(dmrg_heff* H, int32_t precision, int32_t n_vec,
                            const void* psi, void* sigma, void* stream);

/* Allocation-free product, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): dmrg_heff_apply with the partial tiles of split tasks in the
 * library's static device array (256 MiB on each GPU the library runs on,
 * held until the process ends) instead of the context arena, always launched
 * eagerly.  It allocates nothing and calls no allocating routine.  Fails with
 * DMRG_E_WORKSPACE, before any device work, when one vector's partial tiles
 * exceed the array; vectors go in batches of as many as it holds.  Every call
 * on one GPU shares the array (nothing in it must start at zero): calls that
 * overlap on one GPU race.  Arguments and results as dmrg_heff_apply. */
dmrg_status dmrg_heff_apply_static(dmrg_heff* H, int32_t precision, int32_t n_vec, const void* psi, void* sigma,
                                   void* stream);

/* diag[dim] (device, double) = diagonal of H_eff (Davidson preconditioner). */
dmrg_status dmrg_heff_diag(dmrg_heff* H, double* diag, void* stream);

/* Block Davidson for the n_roots lowest eigenpairs of the effective
 * eigenproblem (Appendix A; the paper solves it with Davidson's method).
 * psi_io[n_roots*dim] (device, double): start vectors in, Ritz vectors out.
 * energies[n_roots] host out (e_core included).  Non-convergence is reported
 * in stats, not as an error; DMRG_E_NONFINITE on NaN/Inf in a product. */
dmrg_status dmrg_davidson(dmrg_heff* H, int32_t n_roots, double* psi_io, double* energies,
                          const dmrg_dav_opts* opts, dmrg_dav_stats* stats, void* stream);

/* The same solve one iteration at a time (dmrg_davidson is start, step until
 * done, finish).  start: workspace from the arena, start block psi0 (device,
 * not modified) orthonormalised, first products and Rayleigh-Ritz.  step:
 * one iteration (corrections and their products, or a restart; then
 * Rayleigh-Ritz); *done = 1 once converged, at max_iter / fixed_iters, or
 * when no new direction remains (further steps do nothing); energies
 * [n_roots] (host, optional) receive the current Ritz values and
 * *max_residual (optional) the largest residual norm.  finish: final
 * energies (FP64 Rayleigh quotients when FP32 products were used), Ritz
 * vectors to psi_out[n_roots*dim] (device) and stats.  free releases the
 * workspace (also after a failed call). */
typedef struct dmrg_dav dmrg_dav;
dmrg_status dmrg_davidson_start(dmrg_heff* H, int32_t n_roots, const double* psi0, const dmrg_dav_opts* opts,
                                dmrg_dav** out, void* stream);
dmrg_status dmrg_davidson_step(dmrg_dav* D, int32_t* done, double* energies, double* max_residual);
dmrg_status dmrg_davidson_finish(dmrg_dav* D, double* psi_out, double* energies, dmrg_dav_stats* stats);
void dmrg_davidson_free(dmrg_dav* D);

/* Transformation of the blocked L' = Lb + d1 operators of H through the
 * isometry adding d1 (Appendix A, operator transformation): returns the left
 * block of sites [0, KL+1) in the new renormalized basis.  Reuses the
 * delayed L' operators and integral-weighted sums H already holds. */
dmrg_status dmrg_heff_renormalize(dmrg_heff* H, const dmrg_bsm* isometry, dmrg_opset** out,
                                  void* stream);

/* One blocking + transformation step of any block (Appendix A, blocking
 * formula then operator transformation): `in` grown by its next site (a left
 * block of n sites by site n, a right block of n sites by site K-1-n) and
 * transformed through `isometry` (the MPS tensor of that site; rows in the
 * enlarged order, see the conventions above).  The result holds the same
 * kinds of operators as `in` (normal, or complementary for an NC right
 * block) for the grown block; `in` is left unchanged.  DMRG_E_ARG if the
 * isometry's rows do not match the enlarged sectors. */
dmrg_status dmrg_renormalize(dmrg_ctx* ctx, const dmrg_opset* in, const dmrg_bsm* isometry, dmrg_opset** out,
                             void* stream);

/* Decimation (Appendix A, after the effective eigenproblem): the new
 * renormalized basis of the block that moves on, from the reduced density
 * matrix of the two-site wavefunction.  side DMRG_LEFT: sectors of the
 * enlarged left block L' = Lb + d1 (rows in the enlarged order above; pass
 * the result to dmrg_heff_renormalize or dmrg_renormalize of Lb);
 * DMRG_RIGHT: sectors of R' = d2 + Rb (for dmrg_renormalize of Rb).
 *   psi[n_vec * dim] (device, double; n_vec 1..64): the roots, in H's layout; the density
 *     matrix averages them with equal weights, rho_L = sum_k Psi_k Psi_k^T /
 *     n_vec per sector (rho_R: Psi_k^T Psi_k), Psi_k the wavefunction as a
 *     matrix over (L' state, R' state);
 *   noise, xi: noise >= 0; when noise > 0 the density matrix gains
 *     noise * sum_k Xi_k Xi_k^T / n_vec (Xi_k^T Xi_k on the right), Xi_k the
 *     caller's perturbations (xi[n_vec * dim], device, in H's layout; ignored
 *     when noise == 0): positive semidefinite, independent of the roots' signs;
 *   max_states: M, the states to keep (<= 0: no limit).  Kept are the M
 *     largest weights over all sectors, plus every state within 1e-5 w_M +
 *     1e-12 w_max of the M-th weight w_M (no multiplet of the spin symmetry
 *     is cut), minus every state of weight <= 1e-14 w_max (w_max the
 *     largest weight).
 * The density matrices are GEMMs on the library's FP64 MFMA kernels; each
 * sector's is diagonalised with rocSOLVER (dsyevd), its workspace taken from
 * the arena.  *out: the isometry, columns by descending weight within each
 * sector, sectors without kept states omitted; it lives in the arena until
 * dmrg_iso_free.  info (optional): kept states, sectors, truncation error
 * (discarded / total weight) and total weight.  Synchronizes `stream`.
 * DMRG_E_ARG for bad arguments or a zero wavefunction, DMRG_E_WORKSPACE when
 * the arena cannot hold Psi, the density matrices and the solver workspace,
 * DMRG_E_NONFINITE for a non-finite weight. */
typedef struct dmrg_iso dmrg_iso;
typedef struct {
    int64_t kept;             /* states kept (the new bond dimension) */
    int32_t n_blocks;         /* sectors of the new basis */
    double trunc_err;         /* discarded weight / total weight */
    double weight_total;      /* trace of the density matrix */
} dmrg_decim_info;
dmrg_status dmrg_decimate(dmrg_heff* H, int32_t side, int32_t n_vec, const double* psi, double noise,
                          const double* xi, int32_t max_states, dmrg_iso** out, dmrg_decim_info* info,
                          void* stream);
/* The isometry as a dmrg_bsm (pointers owned by iso, valid until it is freed). */
dmrg_status dmrg_iso_bsm(const dmrg_iso* iso, dmrg_bsm* view);
/* Kept weights (host), block by block in the order of the bsm view,
 * descending within a block; copies min(n, count) and returns the count. */
int64_t dmrg_iso_weights(const dmrg_iso* iso, int64_t n, double* w);
void dmrg_iso_free(dmrg_iso* iso);

/* Arena bytes a call needs (free, beyond what is in use), computed on the
 * host without device work.  what / args:
 *   DMRG_WS_BLOCK       dmrg_ws_block: dmrg_build_block from the vacuum;
 *                       the isometries' metadata only (data may be NULL).
 *                       ctx may be NULL: then K, n_elec, two_sz and the share
 *                       (n_proc, proc_id) come from the args and every
 *                       integral is taken as nonzero (an upper bound);
 *   DMRG_WS_TRANSFORM   dmrg_ws_transform: dmrg_normal_to_complementary;
 *   DMRG_WS_HEFF        dmrg_ws_heff: dmrg_heff_create (default layout);
 *   DMRG_WS_DAVIDSON    dmrg_ws_davidson: dmrg_davidson(_start); ctx may
 *                       be NULL;
 *   DMRG_WS_RENORMALIZE dmrg_ws_renorm: dmrg_renormalize.
 * The build figures are the peak of the smallest batches the build can run
 * in (larger arenas run larger batches); the result of the call (an operator
 * set, an H_eff) is included and stays in the arena afterwards. */
enum { DMRG_WS_BLOCK = 0, DMRG_WS_TRANSFORM = 1, DMRG_WS_HEFF = 2, DMRG_WS_DAVIDSON = 3, DMRG_WS_RENORMALIZE = 4 };
typedef struct {
    int32_t K, n_elec, two_sz, n_proc, proc_id;   /* used when ctx is NULL */
    int32_t side, n_sites, scheme;
    const dmrg_bsm* isometries;
} dmrg_ws_block;
typedef struct { const dmrg_opset* right; } dmrg_ws_transform;
typedef struct { const dmrg_opset* left; const dmrg_opset* right; int32_t n_roots, precision; } dmrg_ws_heff;
typedef struct { int64_t dim; int32_t n_roots; dmrg_dav_opts opts; } dmrg_ws_davidson;
typedef struct { const dmrg_opset* in; const dmrg_bsm* isometry; } dmrg_ws_renorm;
dmrg_status dmrg_query_workspace(const dmrg_ctx* ctx, int32_t what, const void* args, int64_t* bytes);

/* Algorithmic flops of one H_eff psi per vector (sum over terms of the
 * cheaper multiplication order; identity and scalar factors cost 0), and the
 * algorithmic HBM bytes of one product (operators once + psi + sigma). */
int64_t dmrg_heff_flops(const dmrg_heff* H);
int64_t dmrg_heff_bytes(const dmrg_heff* H, int32_t precision);
/* number of H_eff terms (two-index, one-index, block Hamiltonians) */
int32_t dmrg_heff_terms(const dmrg_heff* H, int32_t* n2, int32_t* n1, int32_t* nh);

/* Kernel launches of one H_eff psi product (as dmrg_heff_apply with n_vec =
 * 1), timed one by one with HIP events recorded on `stream` around each
 * launch.  For launch i < n (n >= DMRG_HEFF_LAUNCHES): ms[i] = its duration,
 * flops[i] = the useful MFMA flops of its tiles (2*m*mu*cols per X.U and
 * 2*mu*k*cols per A.B, padding and identities excluded), kind[i] = kernel
 * kind in bits 0-7 (0..5: slice kernel, tiles of 1..6 16-column slices and
 * at most 80 rows; 6..11: the same with at most 96 rows; 12..15: one-wave
 * kernel with (rows, cols) tiles of (16,16), (16,32), (32,16), (32,32);
 * 16..21: tall kernel, tiles of 1..6 slices with 97..320 rows; 22:
 * partial-tile reduction) | 256 when the task records are staged in LDS.
 * Launches with no work report ms = 0.  Synchronizes `stream`.
 * Returns the number of launches (>= 0) or a negative dmrg_status. */
#define DMRG_HEFF_LAUNCHES 23
int32_t dmrg_heff_profile(dmrg_heff* H, int32_t precision, const void* psi, void* sigma, int32_t n, float* ms,
                          double* flops, int32_t* kind, void* stream);

/* Sector metadata of an operator set's basis (host arrays of capacity
 * >= n): returns the sector count; fills qn[2*i], dims[i] when non-null. */
int32_t dmrg_opset_basis(const dmrg_opset* s, int32_t n, int32_t* qn, int64_t* dims);

/* Operator-block readback for tests: copies block (bra sector, ket sector)
 * of the operator named (kind, p, q) into host memory (row-major).  kind:
 * 'H', 'C' (a+_p), 'A' (a+_p a+_q, p<q), 'B' (a+_p a_q), 'R' (R_p), 'Q' (Q_pq),
 * 'D' (P_pq^+, p<q).  Returns DMRG_E_ARG if the operator or block is absent. */
dmrg_status dmrg_opset_block(const dmrg_opset* s, char kind, int32_t p, int32_t q,
                             const int32_t* qn_ket, double* out, int64_t out_elems);

void dmrg_opset_free(dmrg_opset* s);
void dmrg_heff_free(dmrg_heff* H);

#ifdef __cplusplus
}
#endif
#endif
