/*
 * mbbs.h -- C ABI of an MI355X (gfx950) library that solves the Wilson-Dirac
 * equation D X = B for a block of L right-hand sides with the QR-stabilised
 * ("modified") block BiCGSTAB of Nakamura, Ishikawa, Kuramashi, Sakurai and
 * Tadano, right-preconditioned by the Schwarz alternating procedure (SAP).
 *
 * Problem statement (Sec. 2.1): A X = B with A the N x N Wilson-Dirac matrix,
 * N = Lx*Ly*Lz*Lt*3*4, and X, B complex N x L blocks.
 *
 * Conventions shared by every entry point
 *  - Complex numbers are interleaved (re, im) pairs of the stated real type.
 *  - Spinor block layout: row-major N x L with the right-hand side fastest
 *    (Sec. 2.1 keeps the RHS index innermost): element (n, i) sits at
 *    n*L + i, n = 12*site + 3*spin + colour, site = x + Lx*(y + Ly*(z + Lz*t)).
 *  - Gauge layout: U[((site*4 + mu)*3 + a)*3 + b], mu = 0..3 = x,y,z,t;
 *    U_{x,mu} is the link from x to x + mu.
 *  - Gamma matrices: Euclidean chiral basis, gamma_k = [[0, -i s_k], [i s_k, 0]]
 *    (k = 1,2,3 for mu = 0,1,2, s_k Pauli), gamma_4 = [[0, 1], [1, 0]].
 *  - Boundary phases: a hop that wraps forward across x_mu = L_mu - 1 is
 *    multiplied by phase[mu], a backward wrap by its conjugate.
 *  - Pointers named *_dev are device memory (hipMalloc'd or torch tensors on
 *    the current device); everything else is host memory.  `stream` is a
 *    hipStream_t passed as void* (NULL = default stream).
 *  - Return value: 0 = MBBS_OK, 1 = MBBS_NOT_CONVERGED (results valid, tolerance
 *    not reached), < 0 = error; on error nothing was written unless stated,
 *    and mbbs_last_error() holds a message for the calling thread.
 *  - One lattice handle may be used by one stream at a time.
 */
#ifndef MBBS_H
#define MBBS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mbbs_lattice_s* mbbs_lattice_t;

typedef enum {
  MBBS_FP64 = 0,   /* double storage, double arithmetic                         */
  MBBS_FP32 = 1,   /* float storage, float arithmetic                           */
  MBBS_FP16S = 2   /* half storage with one float scale per (site, column),
                      half links, float arithmetic                              */
} mbbs_prec;

enum {
  MBBS_OK = 0,
  MBBS_NOT_CONVERGED = 1,
  MBBS_EINVAL = -1,
  MBBS_ENOMEM = -2,
  MBBS_EHIP = -3,
  MBBS_EBREAKDOWN = -4
};

/* ---------------------------------------------------------------- lattice */

/* Create a lattice: extents dims[4] (all even), SAP domain block[4] (each
 * extent divisible by its block, an even number >= 2 of domains per
 * direction, Sec. 2.2 colours domains even/odd), links U_dev (FP64, layout
 * above, caller keeps ownership; copied), hopping parameter kappa and
 * boundary phases phase[8] = (re, im) per direction, each of modulus 1.
 * The handle owns device copies of the links in FP64/FP32/FP16 in
 * lexicographic and domain-major site order.  Synchronises `stream`.
 * Errors: EINVAL (bad extents, blocks, phases, kappa), ENOMEM, EHIP. */
int mbbs_lattice_create(const int dims[4], const int block[4], const double* U_dev,
                        double kappa, const double phase[8], void* stream,
                        mbbs_lattice_t* out);

/* A batch of nsys independent systems of one shape (dims, block, phases) in
 * one handle, each with its own links U_dev[s] (FP64, layout above, copied)
 * and hopping parameter kappa[s] (host array).  Every kernel launched on the
 * handle serves all of its systems at once: fields hold the systems one
 * after the other (system s occupies rows [s N, (s + 1) N) of an
 * (nsys N) x L block, N = 12 Lx Ly Lz Lt), so the operator, SAP and the
 * solver act on each system exactly as a single-system handle would, while
 * one launch covers every system (the fused form of many small solves).
 * mbbs_solve on a batch handle solves all systems together: B_dev and X_dev
 * are the stacked blocks and `info` points to nsys records; a system that
 * stops early is skipped by every later kernel.  The clover term is not
 * available on batch handles.  Errors as for mbbs_lattice_create.
 * mbbs_lattice_nsys: the number of systems of a handle (1 for a single one). */
int mbbs_lattice_create_batch(int nsys, const int dims[4], const int block[4], const double* const* U_dev,
                              const double* kappa, const double phase[8], void* stream, mbbs_lattice_t* out);
int mbbs_lattice_nsys(mbbs_lattice_t lat, int* nsys);

/* Release every device buffer of the handle.  NULL is accepted. */
int mbbs_lattice_destroy(mbbs_lattice_t lat);

/* Index tables (built on the GPU by the same index functions the kernels
 * use), copied to host memory `out` of `count` int32 entries.
 *  MBBS_TAB_COORD      V x 4   x, y, z, t of each site
 *  MBBS_TAB_NEIGHBOUR  V x 8   column 2mu: site + mu, 2mu+1: site - mu (wrapped)
 *  MBBS_TAB_BOUNDARY   V       bit 2mu+s set if hop (mu, s) wraps the lattice
 *  MBBS_TAB_PARITY     V       (x+y+z+t) mod 2
 *  MBBS_TAB_EO         V       parity*V/2 + site/2
 *  MBBS_TAB_DOMAIN     V       SAP domain id (lexicographic over the domain grid)
 *  MBBS_TAB_COLOUR     V       domain colour, parity of the domain coordinates
 *  MBBS_TAB_LOCAL      V       lexicographic index inside the domain
 *  MBBS_TAB_DM_INDEX   V       position of the site in domain-major order
 *                              (colour-0 domains by id, then colour-1, local inside)
 *  MBBS_TAB_DM_SITE    V       inverse of MBBS_TAB_DM_INDEX
 *  MBBS_TAB_LOCAL_NB   Vb x 8  in-domain neighbour (local index) per hop, -1 if
 *                              the hop leaves the domain
 *  MBBS_TAB_DM_NEIGHBOUR V x 8 neighbours in domain-major positions: row i lists
 *                              the positions of the 8 neighbours of the site at
 *                              position i (what the SAP kernels compute)
 *  MBBS_TAB_HYPERPLANE Vb + nh + 1  SSOR wavefront order: the Vb local indices
 *                              sorted by h = l_0+l_1+l_2+l_3 (ties by local
 *                              index), then the nh + 1 offsets of the
 *                              hyperplanes h = 0 .. nh-1, nh = sum_mu (b_mu - 1) + 1
 * mbbs_lattice_table_size gives the entry count.  Errors: EINVAL. */
enum {
  MBBS_TAB_COORD = 0, MBBS_TAB_NEIGHBOUR, MBBS_TAB_BOUNDARY, MBBS_TAB_PARITY,
  MBBS_TAB_EO, MBBS_TAB_DOMAIN, MBBS_TAB_COLOUR, MBBS_TAB_LOCAL,
  MBBS_TAB_DM_INDEX, MBBS_TAB_DM_SITE, MBBS_TAB_LOCAL_NB, MBBS_TAB_DM_NEIGHBOUR, MBBS_TAB_HYPERPLANE,
  MBBS_TAB_COUNT
};
int mbbs_lattice_table_size(mbbs_lattice_t lat, int which, size_t* count);
int mbbs_lattice_table(mbbs_lattice_t lat, int which, int32_t* out, size_t count);

/* Launch tuning of the stencil kernels (what an autotuner varies).  The
 * operator's output is bit-identical under the group, thread and LDS knobs;
 * the split knob changes the order in which the eight hops are summed, and
 * the SAP domain sums follow the block shape, so those change rounding only
 * (results stay deterministic for a fixed setting).
 * Knobs:
 *  MBBS_TUNE_GROUP_FP64/FP32/FP16S  columns processed per column group by one
 *      pass of blocks over a tile (0 = all L columns; must divide L and be a
 *      multiple of the kernel's columns per thread, else all columns are used)
 *  MBBS_TUNE_BLOCK_THREADS          target threads per block (32..256) of every
 *      precision's stencil kernels
 *  MBBS_TUNE_BLOCK_THREADS_FP64/FP32/FP16S  the same for one precision's kernels
 *      only (the operator and SAP kernels of the other precisions keep theirs)
 *  MBBS_TUNE_SPLIT_FP64/FP32/FP16S  hop groups per site (0 or 1: one thread applies
 *      all 8 hops; 2 or 4: the hops are split over wave-uniform groups that
 *      combine through LDS; falls back to 1 where no launch shape fits)
 *  MBBS_TUNE_PERSIST_BLOCKS         0: one split-wave block per logical block;
 *      1..16: that many resident blocks per CU loop over their XCD's range
 *  MBBS_TUNE_MR_FUSED               SAP domain solver: 1 runs all MR steps of a
 *      colour in one launch, one workgroup per domain (domain-wide sums inside
 *      the workgroup); 0 uses three launches per MR step spread over the whole
 *      chip; -1 (default) picks 1 when a domain holds at most 2048 (site,
 *      column) pairs
 *  MBBS_TUNE_NT_STORE_FP64/FP32/FP16S  1: the operator writes its output with
 *      nontemporal stores (the output is not re-read by the same launch, so it
 *      need not displace neighbour data in L2)
 *  MBBS_TUNE_HOP_PAIR_FP64/FP32/FP16S  1: the one-thread-per-site operator and
 *      SAP residual / MR kernels keep both hops of a direction in flight (more
 *      loads in flight per thread, more registers; 1 or 2 columns per thread)
 *  MBBS_TUNE_CHUNK_FP64/FP32/FP16S  columns per thread of the one-thread-per-site
 *      stencil kernels (0: automatic, 1 for FP64 and 2 otherwise; 1..4 used
 *      when it divides L)
 *  MBBS_TUNE_TILE_FP64/FP32/FP16S   1: the operator (input and output of one
 *      precision) and the MR step's Dirichlet stencil run as LDS-tiled
 *      kernels: one workgroup per sub-block of a SAP domain and all columns,
 *      the sub-block's spinors staged in LDS, only hops leaving it read
 *      global memory (used where a sub-block shape fits; the operator's
 *      output bits are unchanged, the MR sums follow the sub-block shape);
 *      2: as 1, and each MR step also performs the previous step's update of
 *      psi and r (one pass over the fields less per step; same bits as 1);
 *      FP64 and FP32 only (EINVAL for MBBS_TUNE_TILE_FP16S); 3: as 1 with
 *      tiles of at most half the LDS, so two workgroups share a CU (one stages
 *      its tile while the other computes; more hops leave the smaller tile)
 *  MBBS_TUNE_TILE_COLS_FP64/FP32/FP16S  columns per workgroup of the tiled
 *      kernels (0..256; 0, the default: all L): with a value that divides L
 *      into the kernel's column pairs (FP32 / FP16 storage: even) the columns
 *      of a tile are split over L / value adjacent workgroups, each staging
 *      only its columns, so that a larger tile fits the LDS (fewer hops leave
 *      it; its links are read once per workgroup); other values or L act as
 *      0.  Results are the same bits as with 0 for the same tile shape
 *  MBBS_TUNE_MR_ONCE_FP64/FP32/FP16S  1: each MR domain solve of up to 4 steps
 *      forms psi once at its end, psi (+)= c r_0 - sum_j e_j w_j (c = sum_k
 *      omega_k, e_j = omega_j sum_{k>j} omega_k, the same sum as the step-by-step
 *      psi += omega_k r_k regrouped), so that between steps only r is updated:
 *      fewer passes over the fields per domain solve, four more SAP fields in
 *      the workspace (sized while the setting is on; a smaller workspace runs
 *      the step-by-step form); 0 (default): psi updated at every step
 *  MBBS_TUNE_LDS_PAD_KB             extra LDS (KiB, 0..64) reserved per stencil
 *      block, which caps the blocks resident on a CU (fewer sites in flight
 *      per XCD, so more of their neighbour data stays in its L2)
 * Errors: EINVAL for an unknown knob or out-of-range value. */
enum { MBBS_TUNE_GROUP_FP64 = 0, MBBS_TUNE_GROUP_FP32 = 1, MBBS_TUNE_GROUP_FP16S = 2,
       MBBS_TUNE_BLOCK_THREADS = 3, MBBS_TUNE_LDS_PAD_KB = 4, MBBS_TUNE_SPLIT_FP64 = 5,
       MBBS_TUNE_SPLIT_FP32 = 6, MBBS_TUNE_SPLIT_FP16S = 7, MBBS_TUNE_PERSIST_BLOCKS = 8,
       MBBS_TUNE_MR_FUSED = 9, MBBS_TUNE_HOP_PAIR_FP64 = 11, MBBS_TUNE_HOP_PAIR_FP32 = 12,
       MBBS_TUNE_HOP_PAIR_FP16S = 13, MBBS_TUNE_NT_STORE_FP64 = 14, MBBS_TUNE_NT_STORE_FP32 = 15,
       MBBS_TUNE_NT_STORE_FP16S = 16, MBBS_TUNE_CHUNK_FP64 = 17, MBBS_TUNE_CHUNK_FP32 = 18,
       MBBS_TUNE_CHUNK_FP16S = 19, MBBS_TUNE_BLOCK_THREADS_FP64 = 20,
       MBBS_TUNE_BLOCK_THREADS_FP32 = 21, MBBS_TUNE_BLOCK_THREADS_FP16S = 22,
       MBBS_TUNE_TILE_FP64 = 23, MBBS_TUNE_TILE_FP32 = 24, MBBS_TUNE_TILE_FP16S = 25,
       MBBS_TUNE_MR_ONCE_FP64 = 26, MBBS_TUNE_MR_ONCE_FP32 = 27, MBBS_TUNE_MR_ONCE_FP16S = 28,
       MBBS_TUNE_TILE_COLS_FP64 = 29, MBBS_TUNE_TILE_COLS_FP32 = 30, MBBS_TUNE_TILE_COLS_FP16S = 31 };
int mbbs_lattice_tune(mbbs_lattice_t lat, int knob, int value);

/* The tile shape the LDS-tiled kernels use for L columns in precision prec
 * (MBBS_TUNE_TILE_*): t4[0..3] receives the tile extents along x, y, z, t
 * (each dividing the SAP block extent), or zeros when the tiled kernels are
 * not used (knob off, L not split evenly over the kernel's columns per
 * thread, or no tile shape fits the 160 KiB LDS and one workgroup).  t4 is
 * host memory of 4 ints.  Errors: EINVAL. */
int mbbs_lattice_tile_shape(mbbs_lattice_t lat, int L, int prec, int32_t* t4);

/* O(a)-improved (clover) Wilson operator with Jacobi preconditioning (Sec. 2.2:
 * the matrix is divided by I + clover term before the domain decomposition).
 * The clover term, built on the device from the lattice's links and kappa, is
 *   T(x) = i c_sw kappa sum_{mu<nu} sigma_{mu nu} F_{mu nu}(x),
 *   F_{mu nu} = (Q_{mu nu} - Q_{mu nu}^dagger) / 8 (Q: the four plaquettes of
 *   the (mu, nu) plane at x, each traversed mu first), sigma = (i/2)[gamma, gamma];
 * the boundary phases do not enter it.  Once set, every operator of this
 * lattice is A = (1 + T)^{-1} (1 + T - kappa H) = 1 - kappa (1 + T)^{-1} H
 * (mbbs_apply_dirac, the Dirichlet blocks, SAP and SSOR), and mbbs_solve /
 * mbbs_solve_batched solve A X = (1 + T)^{-1} B (residuals refer to that
 * system).  The split-wave kernel shapes are not used with a clover term.
 * mbbs_lattice_set_clover: csw = 0 removes the term.  Errors: EINVAL,
 * ENOMEM, EBREAKDOWN (1 + T singular at a site; the lattice is left without
 * clover term).  Synchronises `stream`.
 * mbbs_lattice_clover_inverse: (1 + T(x))^{-1} as V x 12 x 12 FP64 complex
 * site matrices (row 3*spin + colour) into out_dev (device, V*144 complex).
 * mbbs_apply_clover_inverse: Y = (1 + T)^{-1} X, FP64 N x L device blocks. */
int mbbs_lattice_set_clover(mbbs_lattice_t lat, double csw, void* stream);
int mbbs_lattice_clover_inverse(mbbs_lattice_t lat, double* out_dev, void* stream);
int mbbs_apply_clover_inverse(mbbs_lattice_t lat, int L, const double* X, double* Y, void* stream);

/* ---------------------------------------------------------------- operator */

/* Y = A X with A = 1 - kappa*H, H the hopping term of Sec. 2.1 applied to
 * every one of the L columns with the same links (block hopping-term
 * equation).  X_dev, Y_dev: FP64 N x L blocks (layout above), distinct.
 * prec selects the arithmetic: FP64 directly; FP32 / FP16S convert X to
 * that storage, apply, and convert back (for accuracy checks).  Asynchronous
 * on `stream`.  Errors: EINVAL (L outside 1..256, aliasing, bad prec). */
int mbbs_apply_dirac(mbbs_lattice_t lat, int L, const double* X_dev, double* Y_dev,
                     int prec, void* stream);

/* Same operator on fields already in a precision's own storage (what the
 * solver's kernels see), for timing.  Layout as above with element types:
 *   FP64: double pairs; FP32: float pairs; FP16S: half pairs (X_dev) plus
 *   one float scale per (site, column) at scale[site*L + i] (Xs_dev, Ys_dev).
 * Xs_dev / Ys_dev are ignored unless prec == FP16S. */
int mbbs_apply_dirac_raw(mbbs_lattice_t lat, int L, int prec, const void* X_dev,
                         const float* Xs_dev, void* Y_dev, float* Ys_dev, void* stream);

/* Convert an FP64 N x L block to a precision's storage (RNE) and back. */
int mbbs_convert_to(int prec, size_t nsites, int L, const double* X_dev, void* Y_dev,
                    float* Ys_dev, void* stream);
int mbbs_convert_from(int prec, size_t nsites, int L, const void* X_dev,
                      const float* Xs_dev, double* Y_dev, void* stream);

/* Domain-restricted (Dirichlet) operator, Sec. 2.2: Y = sum_D A_DD X, i.e.
 * A with every hop between two different SAP domains removed, on FP64
 * blocks in lexicographic order, computed in precision `prec`. */
int mbbs_apply_blocked(mbbs_lattice_t lat, int L, const double* X_dev, double* Y_dev,
                       int prec, void* stream);

/* SAP preconditioner, Sec. 2.2: Y = M X with M = K sum_{j<ncy} (1 - A K)^j,
 * K the even-then-odd domain sweep, each domain block approximately inverted
 * by nmr minimal-residual steps from zero (one step size per domain and
 * column).  X_dev, Y_dev: FP64 lexicographic blocks; the preconditioner runs
 * in `prec` in domain-major order; Y is the FP64 image of the result.
 * ws_dev must hold mbbs_sap_workspace_size bytes (caller-owned).  The size
 * depends on the lattice's MBBS_TUNE_TILE_* setting of `prec` (2: two more
 * fields); a workspace sized without it still serves (the MR steps then run
 * unfolded). */
int mbbs_sap_workspace_size(mbbs_lattice_t lat, int L, int prec, size_t* bytes);
int mbbs_sap_apply(mbbs_lattice_t lat, int L, const double* X_dev, double* Y_dev,
                   int ncy, int nmr, int prec, void* ws_dev, size_t ws_bytes, void* stream);

/* SAP with the SSOR domain inverse of Sec. 2.2 (SSOR equations) in place of
 * MR: on each domain A_DD = 1 - Lf - Ub (Lf forward, Ub backward in-domain
 * hops, the paper's L_EE and U_EE) and
 *   B_DD = (1 - w Ub)^{-1} [sum_{j=0}^{nssor} (1 - A^S)^j] (1 - w Lf)^{-1},
 *   A^S = (1/w)[(1 - w Lf)^{-1} + (1 - w Ub)^{-1} + (w - 2)(1 - w Lf)^{-1}(1 - w Ub)^{-1}].
 * The triangular solves run as wavefronts over the hyperplanes
 * l_0+l_1+l_2+l_3 = const of each domain (MBBS_TAB_HYPERPLANE), one
 * workgroup per domain.  nssor is 0 or 1 (the paper uses 1), 0 < omega < 2.
 * mbbs_ssor_workspace_size: device bytes for both calls below.
 * mbbs_sap_apply_ssor: Y = M_SAP X with ncy cycles, as mbbs_sap_apply.
 * mbbs_apply_ssor_blocked: Y = B X with B the block-diagonal SSOR inverse
 * over all domains (both colours).  X, Y: FP64 N x L device blocks, not
 * aliased; prec: storage precision of the sweeps (FP16 storage keeps psi
 * in FP32).  Errors: EINVAL (arguments, workspace), EHIP. */
int mbbs_ssor_workspace_size(mbbs_lattice_t lat, int L, int prec, size_t* bytes);
int mbbs_sap_apply_ssor(mbbs_lattice_t lat, int L, const double* X, double* Y, int ncy, int nssor,
                        double omega, int prec, void* ws, size_t ws_bytes, void* stream);
int mbbs_apply_ssor_blocked(mbbs_lattice_t lat, int L, const double* X, double* Y, int nssor,
                            double omega, int prec, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------ block linear algebra */

/* G = X^H Y, the L x L Gram matrix G[i*L + j] = sum_n conj(X[n,i]) Y[n,j]
 * (steps 4.4, 4.8, 4.11 of Alg. 1 need such products) for FP64 N x L blocks, deterministic fixed-order reduction; G_dev device
 * memory.  ws_dev holds mbbs_gram_workspace_size bytes. */
int mbbs_gram_workspace_size(size_t N, int L, size_t* bytes);
int mbbs_gram(size_t N, int L, const double* X_dev, const double* Y_dev, double* G_dev,
              void* ws_dev, size_t ws_bytes, void* stream);

/* No-allocation form of mbbs_gram, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): same product, same kernels and the same bits as
 * mbbs_gram, with the partial sums kept in a static device buffer the
 * library owns (12 MiB on each device it runs on, held until the process
 * ends) instead of a caller workspace.  L in 1..16 (EINVAL otherwise), any
 * N.  Allocates nothing.  Every call on one device shares that buffer, so
 * calls that overlap on one device (other streams or threads) race; calls in
 * one stream's order do not.  Errors: EINVAL, EHIP. */
int mbbs_gram_noalloc(size_t N, int L, const double* X_dev, const double* Y_dev, double* G_dev,
                      void* stream);

/* Cholesky QR (step 4.1, QR of P): G = P^H P = gamma^H gamma, Q = P gamma^{-1},
 * gamma upper triangular with positive real diagonal (the unique QR factor).
 * passes = 2 repeats the factorisation on Q (CholQR2).  Q_dev may equal P_dev.
 * gamma_dev (L x L, row-major) receives the combined factor.  Returns
 * EBREAKDOWN if P^H P is not numerically positive definite. */
int mbbs_cholqr(size_t N, int L, const double* P_dev, double* Q_dev, double* gamma_dev,
                int passes, void* ws_dev, size_t ws_bytes, void* stream);

/* Solve G X = R for L x L complex G and L x m right-hand sides R (row-major,
 * host or device pointers as named), LU with partial pivoting on
 * |Re|+|Im| (steps 4.4 and 4.11).  Returns EBREAKDOWN on a zero pivot. */
int mbbs_lu_solve(int L, int m, const double* G_dev, const double* R_dev, double* X_dev,
                  void* stream);

/* ---------------------------------------------------------------- solver */

typedef struct {
  double tol;          /* stop when max_i ||r_i||/||b_i|| <= tol (true residual) */
  int maxiter;         /* iteration cap (Alg. 1 loop)                             */
  int max_restarts;    /* restarts from the true residual after a false stop      */
  int ncy;             /* SAP cycles (applications of K)                          */
  int nmr;             /* MR steps per domain                                     */
  int sap_prec;        /* mbbs_prec of the preconditioner                         */
  int x0_is_guess;     /* 1: X_dev holds an initial guess; 0: start from X = 0    */
  int qr_passes;       /* 1 = Cholesky QR, 2 = CholQR2, 0 = no QR step (the plain
                          block BiCGSTAB the paper's QR is measured against)      */
  int graph_iters;     /* iterations per captured HIP graph (0/1: no graph)       */
  int precond;         /* 1: SAP right preconditioner; 0: M = 1                   */
  int memsave;         /* 1: memory-saving form (Alg. 2); 0: Alg. 1               */
  int profile;         /* 1: time kernel classes with HIP events                  */
  int domain_solver;   /* SAP domain solver: 0 = nmr MR steps, 1 = SSOR           */
  int nssor;           /* SSOR correction terms N_SSOR (0 or 1)                   */
  double ssor_omega;   /* SSOR relaxation, 0 < omega < 2                          */
  const double* rtilde;/* R~ of Alg. 1 (its choice is left open): a device FP64 N x L block
                          (a batch handle: the systems' blocks stacked), read
                          once at the start; NULL: R~ = R_0                       */
} mbbs_solve_params;

/* Kernel classes timed when params.profile = 1. */
enum { MBBS_K_DSLASH64 = 0, MBBS_K_SAP_RES, MBBS_K_MR_DSLASH, MBBS_K_MR_UPDATE,
       MBBS_K_CONVERT, MBBS_K_GRAM, MBBS_K_UPDATE, MBBS_K_SMALL, MBBS_K_SSOR, MBBS_K_COUNT };

typedef struct {
  int status;                   /* return value of the call                        */
  int iterations;               /* Alg. 1 iterations performed                     */
  int restarts;
  long long n_dslash_outer;     /* full-lattice FP64 applications of A             */
  long long n_sap;              /* applications of M                               */
  double* true_res;             /* caller-owned host arrays of length L: final      */
  double* rec_res;              /* ||b - A x||/||b|| and recursive ||r||/||b||      */
  double seconds;               /* wall time of the call                           */
  double kernel_ms[MBBS_K_COUNT];        /* summed kernel time per class (profile) */
  long long kernel_launches[MBBS_K_COUNT];
  double* res_history;          /* caller-owned host array of history_cap doubles, or
                                   NULL: max_i ||r_i||/||b_i|| of the recursive residual
                                   after each iteration (Sec. 3.3, residual against
                                   iterations); at most 4096 entries are kept        */
  int history_cap;
  int history_len;              /* entries written (iterations, capped)            */
} mbbs_solve_info;

void mbbs_solve_params_default(mbbs_solve_params* p);

/* Workspace (device bytes) needed by mbbs_solve for this lattice, L, params. */
int mbbs_solve_workspace_size(mbbs_lattice_t lat, int L, const mbbs_solve_params* params,
                              size_t* bytes);

/* Solve A X = B (Alg. 1, or Alg. 2 if params->memsave): B_dev, X_dev FP64
 * N x L blocks; X_dev is read as the initial guess when x0_is_guess and
 * always receives the result.  R~ = R_0 unless params->rtilde supplies it.
 * The loop test (continue while max_i ||r_i||/||b_i|| > tol) runs on the
 * device on R_0 and after step 4.10 of every iteration; once the recursion
 * stops, the FP64 true residual B - A X is formed, and if it is above tol the
 * iteration restarts from R = B - A X, P = R, keeping R~ (at most
 * max_restarts times).  The outer recurrences, Gram
 * products, Cholesky QR, L x L solves and the true residual run in FP64;
 * SAP runs in params->sap_prec.  Allocates nothing: ws_dev (caller-owned,
 * mbbs_solve_workspace_size bytes) holds every intermediate.  Blocks until
 * done.  Returns OK, NOT_CONVERGED (maxiter or restarts exhausted; X and
 * residuals valid), EBREAKDOWN (singular R~^H V, non-positive P^H P or
 * non-finite coefficient; X is the last consistent iterate), EINVAL (bad
 * arguments, a zero column of B, workspace too small). */
int mbbs_solve(mbbs_lattice_t lat, int L, const double* B_dev, double* X_dev,
               const mbbs_solve_params* params, void* ws_dev, size_t ws_bytes,
               mbbs_solve_info* info, void* stream);

/* Solve nsys independent jobs (each its own lattice handle, L, B, X and
 * params) together.  A job on a batch handle (mbbs_lattice_create_batch)
 * covers all of that handle's systems in fused launches (stacked B and X);
 * `infos` holds one record per system, the jobs' systems in argument order.
 * The jobs are spread over up to 4 internal streams (created and destroyed
 * by the call, default priority; the first waits for the work already on
 * `stream`), largest first onto the least loaded one, so the launches of
 * small jobs run concurrently.  Each job advances in batches of graph_iters
 * iterations (captured once in a per-job HIP graph and replayed when
 * graph_iters > 1); the host polls one event per job and enqueues its next
 * batch, true-residual check or restarts as soon as its previous batch has
 * drained, without waiting for the other jobs.  A system that converges
 * inside a batch stops on a device flag.  ws_dev holds
 * mbbs_solve_batched_workspace_size bytes (device); the call also takes small
 * pinned host buffers for the state records.  Blocks until every system is
 * done; each record and the return value are as for mbbs_solve (the worst
 * status over the systems). */
int mbbs_solve_batched_workspace_size(int nsys, const mbbs_lattice_t* lats, const int* Ls,
                                      const mbbs_solve_params* params, size_t* bytes);
int mbbs_solve_batched(int nsys, const mbbs_lattice_t* lats, const int* Ls,
                       const double* const* B_dev, double* const* X_dev,
                       const mbbs_solve_params* params, void* ws_dev, size_t ws_bytes,
                       mbbs_solve_info* infos, void* stream);

/* Message of the last failed call on this thread ("" if none). */
const char* mbbs_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MBBS_H */
