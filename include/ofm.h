/*
 * ofm.h -- C ABI of the overlapping-fragments-method (OFM) library for AMD
 * Instinct MI355X (gfx950).
 *
 * The method (Vukmirovic & Wang, "Overlapping fragments method for electronic
 * structure calculation of large systems", Sec. II) represents the
 * single-particle Hamiltonian H = -1/2 Laplacian + V (Eq. 1) in the basis of
 * the lowest eigenstates of many mutually overlapping fragments.  The library
 * computes, on one GPU:
 *
 *   1. ofm_build_fragments  -- fragment boxes, the pair list and the potential
 *                              restricted to every box;
 *   2. ofm_solve_fragments  -- the lowest s_j eigenpairs of every fragment
 *                              Hamiltonian (one batched eigensolver for all
 *                              fragments) and H|phi> with the Hamiltonian of
 *                              the entire system, as the matrix elements
 *                              need (Sec. II);
 *   3. ofm_matrix_elements  -- H_{ij,mn} = <phi_i^(j)|H|phi_m^(n)> and
 *                              S_{ij,mn} = <phi_i^(j)|phi_m^(n)> for every
 *                              overlapping pair (Sec. II);
 *   4. ofm_solve_global     -- the generalised eigenproblem
 *                              sum_mn (H - E S) C = 0 (Eq. 2).
 *
 * Discretisation (the paper's plane-wave basis is replaced by a real-space
 * grid): uniform spacing h, x-fastest point order (index = x + nx*(y +
 * ny*z)), 4th-order central second difference, Dirichlet walls one spacing
 * outside every box (global grid and fragments alike) with odd-image second
 * ghosts.  Inner products are plain l2 sums over grid points; every returned
 * state has sum phi^2 = 1.  Units are Hartree atomic units.
 *
 * Conventions for every call:
 *  - Return value is an ofm_status; nothing else crosses the ABI (no C++
 *    exceptions, no abort).  On error, ofm_last_error(ctx) returns a message.
 *  - Buffers named "host" are caller-owned host memory; the library copies
 *    from / to them before returning.  Buffers named "host or device" may be
 *    either; device pointers are borrowed only for the duration of the call.
 *  - The library owns ofm_ctx / ofm_frags / ofm_mats handles; free them with
 *    the matching *_destroy call.  Sizes for output buffers come from
 *    ofm_frags_info / ofm_fragment_geometry (two-call pattern).
 *  - All device work is enqueued on the context stream; every call that
 *    returns results on the host synchronises that stream first.  A context
 *    and the handles made with it must be used by one host thread at a time;
 *    different contexts may be driven from different threads at once (the
 *    library serialises its stream captures with its rocBLAS / rocSOLVER
 *    calls, which may not overlap across threads).
 *  - The precision form is fixed when the context is created.
 */
#ifndef OFM_H
#define OFM_H

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  OFM_OK = 0,
  OFM_E_INVALID = -1,   /* bad argument: NaN/Inf in V, box outside the grid,
                           s_j > n_j, NULL where a buffer is required, ...   */
  OFM_E_NOMEM = -2,     /* device or host allocation failed                  */
  OFM_E_DEVICE = -3,    /* a HIP / rocSOLVER / rocBLAS call failed           */
  OFM_E_NOCONV = -4,    /* eigensolver hit max_iter; results are returned and
                           the per-fragment converged flags say which        */
  OFM_E_SINGULAR = -5,  /* every eigenvalue of S is below the threshold      */
  OFM_E_STATE = -6      /* call out of order (e.g. elements before states)   */
} ofm_status;

typedef enum {
  OFM_FP64 = 0,          /* all vector arithmetic and products in FP64       */
  OFM_MIXED_BF16X3 = 1,  /* vectors and stencil in FP32; the Rayleigh-Ritz
                            and element contractions as 3-term split-BF16
                            MFMA products (a_hi b_hi + a_hi b_lo + a_lo b_hi)
                            with FP32 sums over at most a few hundred points
                            added in FP64; CholQR Gram (FP64 products),
                            Cholesky, small eigensolves and the global solve
                            in FP64                                          */
  OFM_MIXED_FP16X3 = 2   /* as OFM_MIXED_BF16X3 with the split in FP16:
                            a_hi = f16(a), a_lo = f16((a - a_hi) 2^11), the
                            cross products scaled back by 2^-11 (dropped term
                            ~2^-22 |a b| against ~2^-16 for BF16)           */
} ofm_precision;

/* Global grid: point (ix,iy,iz) at origin + (ix,iy,iz)*h (bohr). */
typedef struct {
  int nx, ny, nz;
  double h;
  double origin[3];
} ofm_grid;

/* One fragment: a cuboid box of grid points [lo, lo+dims) in global indices
   (x, y, z order) and the number of its lowest states kept in the basis. */
typedef struct {
  int lo[3];
  int dims[3];
  int n_states;
} ofm_fragment_desc;

/* Eigensolver options.  Fields set to 0 take the default in brackets. */
typedef struct {
  double tol;            /* residual bound ||H_j phi - eps phi||_2 per wanted
                            state [1e-10 FP64, 2e-5 mixed]                   */
  int max_iter;          /* outer (filter + Rayleigh-Ritz) iterations [60]   */
  int guard;             /* extra block vectors beyond s_j [6]               */
  int degree;            /* Chebyshev filter degree per iteration, rounded
                            up to even [42 FP64, 36 mixed]                   */
  unsigned long long seed; /* start-vector seed [0]                          */
  int use_graph;         /* >= 0: the Chebyshev filter sweep is captured once
                            as a HIP graph and replayed every iteration [on];
                            -1: launch its kernels one by one               */
  int autotune;          /* >= 0: time the variants of the strip stencil
                            on the strips of the first filter sweep (boxes
                            outside the multi-step classes; none: nothing
                            is timed), once per (precision, largest box
                            plane) and context, and keep the fastest, which
                            also runs H X in FP64 [on]; -1: use the fixed
                            default variant                                */
  int resident;          /* >= 0: in the mixed form, boxes of at most 32
                            points per axis run the whole filter in one
                            launch with the vector held on chip (same bits
                            as the per-step launches) [on]; -1: per-step
                            launches for every box                         */
  int fused;             /* filter steps per launch for the boxes whose xy
                            plane holds at most 2048 points in FP64, 3072
                            in the mixed forms (larger planes run one step
                            per launch): 0 or 3: three
                            [default]; 2: two; -1 (or 1): one.  Same bits in
                            every case.                                    */
} ofm_solve_opts;

typedef struct ofm_ctx ofm_ctx;
typedef struct ofm_frags ofm_frags;
typedef struct ofm_mats ofm_mats;

/* ---- context ---------------------------------------------------------- */

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t to
   enqueue on (borrowed, must outlive the context) or NULL for a stream owned
   by the context. */
ofm_status ofm_create(ofm_ctx** ctx, int device, void* hip_stream,
                      ofm_precision precision);
/* Returns OFM_E_STATE (and destroys nothing) while fragment or matrix
   handles made with ctx are still alive. */
ofm_status ofm_destroy(ofm_ctx* ctx);
/* Message for the last failed call on ctx (owned by ctx; "" if none).
   ctx may be NULL for errors of ofm_create itself. */
const char* ofm_last_error(const ofm_ctx* ctx);
/* Library version string (static storage). */
const char* ofm_version(void);

/* ---- fragments (Sec. II: fragments are boxes; Sec. III-C: pair set) ---- */

/* Set up fragments on the grid.
   V        : potential, nx*ny*nz doubles, x fastest (host or device).
   frags    : n_frag descriptors (host).
   atom_xyz, frag_atom_ptr, frag_atom_idx: optional atom positions (3*n_atoms
              doubles, bohr) and CSR lists of each fragment's atoms (host);
              only used when d_cut > 0.
   d_cut    : <= 0 selects the exact pair set of the stencil: {j,n} is a pair
              iff box_j grown by the stencil reach (2 points) meets box_n, and
              every dropped block is exactly zero.  > 0 additionally drops
              pairs whose closest atoms are >= d_cut apart (Sec. III-C).
   Errors: OFM_E_INVALID for a box outside the grid, dims < 1, n_states < 1
   or > box points, non-finite V or h <= 0. */
ofm_status ofm_build_fragments(ofm_ctx* ctx, const ofm_grid* grid,
                               const double* V, int n_frag,
                               const ofm_fragment_desc* frags,
                               const double* atom_xyz,
                               const long long* frag_atom_ptr,
                               const int* frag_atom_idx, double d_cut,
                               ofm_frags** out);
ofm_status ofm_frags_destroy(ofm_frags* f);
/* Sizes: basis size sum_j s_j, number of stored blocks (pairs j<=n,
   diagonal included) and sum_j n_j.  Any pointer may be NULL. */
ofm_status ofm_frags_info(const ofm_frags* f, long long* n_basis,
                          long long* n_pairs, long long* total_points);
/* Geometry of fragment j: its box, its dilated box (box grown by 2 points per
   side, clipped to the grid: the support of H|phi>), and s_j.  Any output
   pointer may be NULL. */
ofm_status ofm_fragment_geometry(const ofm_frags* f, int j, int lo[3],
                                 int dims[3], int dlo[3], int ddims[3],
                                 int* n_states);
/* The pair list (j <= n) in storage order, and the offset of each block in
   the packed block arrays (block p is s_j x s_n row-major at block_off[p]).
   Arrays sized n_pairs (host). */
ofm_status ofm_pairs(const ofm_frags* f, int* pair_j, int* pair_n,
                     long long* block_off);

/* ---- fragment eigenstates (Sec. II, Sec. III-B) ------------------------- */

/* Lowest s_j eigenpairs of every fragment Hamiltonian H_j (V restricted to
   box j, walls at the box faces), all fragments in one batched solver, then
   H|phi> with the whole-system H on every dilated box.
   eps       : sum_j s_j doubles, fragment by fragment (host, may be NULL).
   iters     : n_frag ints, outer iterations used (host, may be NULL).
   converged : n_frag bytes, 1 if every wanted residual <= tol (host, may be
               NULL).
   Returns OFM_E_NOCONV (results still valid) if any fragment missed tol. */
ofm_status ofm_solve_fragments(ofm_ctx* ctx, ofm_frags* f,
                               const ofm_solve_opts* opts, double* eps,
                               int* iters, unsigned char* converged);
/* Per-fragment flags of the last ofm_solve_fragments (n_frag ints, host):
   bit 0 -- the Cholesky factorisation of a CholQR Gram matrix lost a pivot
            and the shifted factorisation (G + 1e-12 b_j I after unit-diagonal
            scaling) was used at least once;
   bit 1 -- the shifted factorisation lost a pivot as well (the block was
            numerically rank deficient); such a fragment is reported as not
            converged and the solve returns OFM_E_NOCONV.
   All zero before the first solve.  Errors: OFM_E_INVALID for NULL. */
ofm_status ofm_solve_flags(const ofm_frags* f, int* flags);
/* States of fragment j: phi is s_j*n_j doubles, state-major (state i at
   phi + i*n_j, points x fastest); eps is s_j doubles.  Host.  Sign gauge:
   the largest-|.| component of every state is positive (first on ties). */
ofm_status ofm_get_states(const ofm_frags* f, int j, double* phi, double* eps);
/* Import states for fragment j (same layout; host), e.g. to evaluate matrix
   elements for externally computed states or to resume.  The whole-system
   H|phi> is recomputed for j.  Rows are used as given (no orthonormalisation):
   S_jj of an imported fragment is computed from its states in both forms
   (in the mixed form with FP64 products on the FP32-stored states), whereas
   the mixed form takes S_jj = I for states that ofm_solve_fragments
   orthonormalised in FP64. */
ofm_status ofm_set_states(ofm_frags* f, int j, const double* phi,
                          const double* eps);
/* H|phi> of fragment j with the whole-system H on its dilated box: s_j *
   (ddims product) doubles, state-major, x fastest (host). */
ofm_status ofm_get_hphi(const ofm_frags* f, int j, double* hphi);
/* Apply the fragment Hamiltonian H_j to nvec vectors of box j (state-major,
   host in and out): the stencil of the eigensolver, exposed for checking.
   Errors: OFM_E_INVALID for nvec outside [1, OFM_MAX_APPLY_VECTORS], j out
   of range or a NULL buffer (no device work is done then). */
#define OFM_MAX_APPLY_VECTORS 32767
ofm_status ofm_apply_fragment_h(ofm_ctx* ctx, ofm_frags* f, int j, int nvec,
                                const double* x, double* y);

/* Build every fragment Hamiltonian from the wells of the fragment's own
   atoms instead of the global V restricted to the box (the paper builds the
   fragment Hamiltonian from the fragment's own charge density, Sec. II):
   V_j(r) = sum_{a in fragment j} -Z_a exp(-|r - R_a|^2 / (2 sigma^2)) for
   |r - R_a| < r_cut, at the box's grid points (origin + index * h).
   H|phi> keeps the whole-system V given to ofm_build_fragments.
   atom_xyz: 3*n_atoms doubles; Z: n_atoms; frag_atom_ptr: n_frag + 1;
   frag_atom_idx: the atoms of each fragment (all host).  Call before
   ofm_solve_fragments; states computed earlier are not recomputed.
   Errors: OFM_E_INVALID for sigma or r_cut <= 0, non-finite inputs, or an
   atom index outside [0, n_atoms). */
ofm_status ofm_set_fragment_wells(ofm_frags* f, int n_atoms,
                                  const double* atom_xyz, const double* Z,
                                  double sigma, double r_cut,
                                  const long long* frag_atom_ptr,
                                  const int* frag_atom_idx);

/* Pin the stencil variant used for fragments f (0..2: 256, 512, 1024 plane
   points per workgroup in FP64; 512, 1024, 2048 in the mixed form), or -1 to
   let ofm_solve_fragments pick by timing the variants (the default).  Every
   variant computes identical values. */
ofm_status ofm_set_stencil_variant(ofm_frags* f, int variant);

/* Pin the variant of the pair-contraction kernels for calls on ctx (0: a
   chunk of the overlap is loaded and then multiplied; 1: the next chunk's
   loads stay in flight during the products), or -1 to let the first
   ofm_matrix_elements call per (precision, block-width class) time both and
   keep the faster (the default; the choice is cached in ctx).  Every variant
   computes identical values. */
ofm_status ofm_set_pair_variant(ofm_ctx* ctx, int variant);

/* ---- matrix elements (Sec. II) ------------------------------------------ */

/* H and S blocks for every pair j <= n: S_jn = Phi_j^T Phi_n over box_j ^
   box_n, H_jn = Phi_j^T (H Phi_n) over box_j ^ dil(box_n); diagonal blocks
   are symmetrised.  One grouped launch for all pairs.  Requires states
   (ofm_solve_fragments or ofm_set_states for every fragment). */
ofm_status ofm_matrix_elements(ofm_ctx* ctx, ofm_frags* f, ofm_mats** out);
/* Number of stored doubles per matrix (sum over pairs of s_j*s_n). */
ofm_status ofm_mats_info(const ofm_mats* m, long long* n_values);
/* Copy the packed blocks (layout of ofm_pairs) to host buffers of
   n_values doubles each; either pointer may be NULL. */
ofm_status ofm_mats_copy(const ofm_mats* m, double* H_blocks,
                         double* S_blocks);
ofm_status ofm_mats_destroy(ofm_mats* m);

/* ---- generalised eigenproblem (Eq. 2) ----------------------------------- */

/* Solve sum_mn (H - E S) C = 0 in the fragment basis, FP64 on the GPU:
   S = U diag(s) U^T; directions with s < s_thresh are dropped; X =
   U_K diag(s_K^-1/2); eigenpairs of X^T H X.  Eigenvalues in [e_lo, e_hi]
   are returned ascending.
   n_kept : |K| (host, may be NULL).   n_eig : number written to E (host).
   E      : capacity n_basis doubles (host).
   C      : optional, n_basis * n_eig doubles, column k (stride n_basis) the
            coefficients of eigenvalue k (host, may be NULL).
   s_min  : smallest kept eigenvalue of S (host, may be NULL).
   Returns OFM_E_SINGULAR if no eigenvalue of S reaches s_thresh. */
ofm_status ofm_solve_global(ofm_ctx* ctx, const ofm_mats* m, double s_thresh,
                            double e_lo, double e_hi, int* n_kept, int* n_eig,
                            double* E, double* C, double* s_min);

/* ---- basis near the fragment HOMOs and the HOMO-LUMO gap (Sec. III-B) --- */
/* The computed states of a fragment play the role of its occupied states;
   the highest one is its HOMO. */

/* Keep mask over the basis (fragment by fragment in basis order, n_basis
   bytes, host) from the fragment eigenvalues of the last
   ofm_solve_fragments (or imported states).  For each fragment, walk down
   from its HOMO and keep the states above the first gap
   eps[k] - eps[k-1] >= gap_min found among its top n_max states; with no
   such gap, or gap_min <= 0, keep its top n_max states (all of them where
   s_j <= n_max).  Errors: OFM_E_INVALID for n_max < 1; OFM_E_STATE without
   states. */
ofm_status ofm_select_homo(const ofm_frags* f, int n_max, double gap_min,
                           unsigned char* keep);

/* ofm_solve_global on the pencil restricted to the basis functions with
   keep[i] != 0 (n_basis bytes, host; NULL keeps every function).  Rows of C
   follow the kept functions in basis order (n_sel rows, column stride
   n_sel).  Errors as ofm_solve_global, and OFM_E_INVALID when nothing is
   kept. */
ofm_status ofm_solve_global_subset(ofm_ctx* ctx, const ofm_mats* m,
                                   const unsigned char* keep,
                                   double s_thresh, double e_lo, double e_hi,
                                   int* n_kept, int* n_eig, double* E,
                                   double* C, double* s_min);

/* ---- windowed solve of a large basis (Sec. II, Sec. III-D) -------------- */

/* Keep mask (n_basis bytes, host, fragment by fragment in basis order) of the
   basis functions whose fragment eigenvalue lies in [e_lo, e_hi] (inclusive),
   from the last ofm_solve_fragments (or imported states).
   Errors: OFM_E_INVALID for a NULL mask or non-finite bounds; OFM_E_STATE
   without states. */
ofm_status ofm_select_band(const ofm_frags* f, double e_lo, double e_hi,
                           unsigned char* keep);

/* Eigenvalues of Eq. 2 in the window [e_lo, e_hi] for a basis too large for
   the dense pencil: the pencil is restricted to the basis functions whose
   fragment eigenvalue lies within a margin of the window (ofm_select_band
   on [e_lo - margin, e_hi + margin]), solved as ofm_solve_global_subset
   (threshold s_thresh).  Round r uses the margin margin0 + r * margin_step,
   r < max_rounds; a round whose band holds no more functions than the last
   one solved is skipped.  The window has converged when two successive
   solved bands give the same number of window eigenvalues, equal within tol
   (Ha), or when a band holds the whole basis (that round is the full
   ofm_solve_global_subset of every function).  This is a reduction of the
   basis, not an exact solve of the whole pencil: the omitted functions
   shift the window's eigenvalues at second order in their coupling, which
   the convergence test bounds only empirically.
   n_eig  : eigenvalues written to E (capacity n_basis), ascending.
   margin : margin of the last round (host, may be NULL).
   n_sel  : basis functions of the last round's pencil (host, may be NULL).
   n_kept : kept directions of S in the last round (host, may be NULL).
   Returns OFM_E_NOCONV (last round's eigenvalues returned) when max_rounds
   pass without two agreeing rounds.  Errors: OFM_E_INVALID for
   margin0 < 0, margin_step <= 0, max_rounds < 2, tol < 0, e_hi < e_lo or
   non-finite arguments, and as ofm_solve_global_subset. */
ofm_status ofm_solve_global_window(ofm_ctx* ctx, const ofm_mats* m,
                                   double s_thresh, double e_lo, double e_hi,
                                   double margin0, double margin_step,
                                   int max_rounds, double tol, int* n_eig,
                                   double* E, double* margin, long long* n_sel,
                                   int* n_kept);

/* The dense FP64 symmetric eigensolver behind ofm_solve_global (it
   diagonalises S and H' of the canonical orthogonalisation that solves
   Eq. 2), for callers with a pencil of their own.  A: n*n doubles, host,
   column-major, symmetric (both triangles are read; they should agree).
   w: n doubles, host, the eigenvalues in ascending order.  Z: NULL, or n*n
   doubles, host, column k the unit eigenvector of w[k] (each column's sign
   is arbitrary).  Device memory, freed on return: two copies of A (one
   with its leading dimension rounded up to 64), with Z also Z and
   rocSOLVER's divide-and-conquer workspace, and from n = 2049 on the tiled
   product's partial sums, (n/256 + n/32 + 2) n doubles (about 1/29 of A).
   Errors:
   OFM_E_INVALID for n < 1, n > 65536, a NULL A or w, or a NaN or Inf in A;
   OFM_E_DEVICE when the tridiagonal solver does not converge;
   OFM_E_NOMEM. */
ofm_status ofm_dense_eigh(ofm_ctx* ctx, int n, const double* A, double* w,
                          double* Z);

/* e_j = <HOMO_j|H|HOMO_j> with the whole-system H for every fragment, read
   from the diagonal blocks of m (n_frag doubles, host). */
ofm_status ofm_homo_energies(const ofm_mats* m, double* e);

/* First gap above e_ref in the spectrum E[0..n) (ascending, host): scanning
   upward from the first eigenvalue >= e_ref, the first spacing
   E[k+1] - E[k] >= gap_min.  Writes n_occ = k + 1 (states up to the gap are
   occupied), e_homo = E[k], e_lumo = E[k+1]; n_occ = -1 and NaN energies
   when there is no such gap.  Errors: OFM_E_INVALID for n < 0, a NULL
   output, non-finite e_ref or gap_min < 0, or E not ascending. */
ofm_status ofm_homo_lumo_gap(const double* E, int n, double e_ref,
                             double gap_min, int* n_occ, double* e_homo,
                             double* e_lumo);

/* ---- measurement -------------------------------------------------------- */

/* Turn per-launch HIP-event timing of the library's kernels on or off.  When
   on, the library records an event pair around each launch of the timed
   kernels on the context stream. */
ofm_status ofm_set_profiling(ofm_ctx* ctx, int on);
/* Accumulated timing of one kernel family since the last reset: "stencil"
   (one fragment-Hamiltonian step per launch), "multistep" (two or three
   filter steps per launch), "filter" (whole filter with the vector on chip), "gram"
   (subspace contractions), "elements" (pair contractions), "rotate",
   "tridiag" (one whole tridiagonal reduction of the dense eigensolver per
   entry; its bytes are the trailing-matrix stream of its column products).
   total_ms is the sum of launch durations, alg_bytes the algorithmic HBM
   bytes of those launches (inputs read once, outputs written once), flops
   their useful flops. */
ofm_status ofm_kernel_stats(ofm_ctx* ctx, const char* family,
                            long long* launches, double* total_ms,
                            double* alg_bytes, double* flops);
ofm_status ofm_reset_stats(ofm_ctx* ctx);
/* Wall time (ms, host clock around the call) of the last solve_fragments,
   matrix_elements and solve_global calls. */
ofm_status ofm_stage_times(const ofm_ctx* ctx, double* solve_ms,
                           double* elements_ms, double* global_ms);

/* ---- allocation-free matrix elements ------------------------------------ */

/* Bytes of the per-GPU device array that ofm_matrix_elements_noalloc stages
   its pair task list in (one array per GPU the library runs on, held until
   the process ends): 64 MiB, i.e. up to about 5.5e5 tasks (two per pair of
   fragments at most). */
#define OFM_NOALLOC_SCRATCH_BYTES (64LL << 20)

/* For callers that cannot allocate device memory (code under HIP stream
   capture, tight serving loops, harnesses that forbid hipMalloc): the work
   of ofm_matrix_elements written into caller-owned device buffers, with no
   device allocation and no allocating library call.
   H_dev, S_dev : device pointers to n_values doubles each, where n_values =
                  sum over pairs of s_j * s_n (block_off[last] + s_j * s_n of
                  the last pair of ofm_pairs); the blocks are written in the
                  layout of ofm_pairs (and ofm_mats_copy), every element,
                  blocks without overlap as zeros.
   The pair task list is copied from the host into the library's scratch
   array (OFM_NOALLOC_SCRATCH_BYTES, resolved per device by ofm_create).  The
   work is enqueued on the context stream and the call returns without
   waiting for it: synchronise that stream before reading H_dev / S_dev.
   Every call on one GPU shares that GPU's scratch array and the array keeps
   the last call's task list: calls whose work overlaps on one GPU (contexts
   on different streams of the same device with calls in flight at once)
   race on it; calls ordered on one stream do not.  Per-kernel timing
   (ofm_set_profiling) is not recorded for this call.
   Errors: OFM_E_INVALID for a NULL handle or buffer, a buffer that is not
   device memory, or a task list larger than the scratch array (nothing is
   enqueued then); OFM_E_STATE without states. */
ofm_status ofm_matrix_elements_noalloc(ofm_ctx* ctx, ofm_frags* f,
                                       double* H_dev, double* S_dev);

#ifdef __cplusplus
}
#endif
#endif /* OFM_H */
