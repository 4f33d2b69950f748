/*
 * mgic.h - C ABI of the MI355X (gfx950) adaptive-multigrid / LPT library.
 *
 * What it computes (Hahn & Abel 2011, "Multi-scale initial conditions for
 * cosmological simulations"):
 *   - the potential phi of Poisson's equation  L phi = f  on a periodic base
 *     grid and on nested 2x zoom-in patches, by the FAS multigrid V-cycle of
 *     Section 3.2 (red-black Gauss-Seidel, nu1 = nu2 = 2, 8-child mean
 *     restriction, injection prolongation) extended to nested sub-grids as in
 *     Section 3.3 (ghost zones by quadratic interpolation parallel then
 *     normal to the coarse-fine face, flux matching with Table 2's order-1
 *     flux operator);
 *   - first-order (Zel'dovich) displacements  psi = scale * G phi  with the
 *     fourth- or sixth-order gradient G of Table 1 (Section 3.1, eq. "zeldovich");
 *   - the second-order source  tau = sum_{i>j} (D_ii D_jj - D_ij^2),
 *     D_ij = G_i G_j phi  (Section 3.1, second-order perturbations), whose
 *     Poisson solve gives the second-order potential.
 *
 * Conventions shared by every entry point
 *   - All field pointers are DEVICE pointers to float64 arrays laid out
 *     row-major [nx][ny][nz] (z contiguous), without ghost padding.
 *   - Level 0 of a hierarchy is the periodic base (cubic, n^3 cells, spacing
 *     h).  Level p >= 1 is a patch of n[0] x n[1] x n[2] cells (each even,
 *     >= 4) of spacing h_{p-1} / 2 whose first cell is the first child of
 *     cell off[] of level p-1.  A patch in the base must not wrap and must
 *     leave >= 2 base cells uncovered per axis; a patch in a patch keeps >= 4
 *     parent cells from its parent's faces.
 *   - The caller owns every buffer (inputs, outputs, workspace).  The library
 *     never allocates device memory on these paths: it carves the caller's
 *     workspace (size from the matching *_workspace_bytes query, any
 *     256-byte-aligned device buffer of at least that size).
 *   - `stream` is a hipStream_t (NULL = the default stream).  Work is
 *     enqueued on it; calls that need a host decision (per-cycle convergence
 *     test) synchronise that stream, others are asynchronous.
 *   - Return value: MG_OK (0) or a negative MG_E* code; mg_last_error()
 *     returns a human-readable message for the calling thread.
 */
#ifndef MGIC_H
#define MGIC_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MG_MAX_LEVELS 8

enum {
    MG_OK = 0,
    MG_EINVAL = -1,     /* bad argument: null pointer, size, nesting, workspace too small   */
    MG_ENOCONV = -2,    /* max_cycles reached above tol: u holds the last iterate           */
    MG_EDIVERGED = -3,  /* NaN/Inf residual or growth over 3 consecutive cycles             */
    MG_EHIP = -4        /* HIP runtime error                                                 */
};

/* precision of the smoother / transfer operators */
enum { MG_FP64 = 0, MG_MIXED = 1 };

/* option flags */
#define MG_USE_INITIAL_GUESS 0x1u  /* start from the caller's u instead of 0                    */
#define MG_FIXED_CYCLES      0x2u  /* run exactly max_cycles cycles, no per-cycle host readback */
/* Graph capture: mg_solve_level, mg_solve_hierarchy and mg_solve_hierarchy_noalloc may be called
 * on a stream that the caller is capturing into a HIP graph, with MG_FIXED_CYCLES (without it
 * they return MG_EINVAL before any device work: a converging solve reads its residual back).
 * They then launch their kernels into the capture, replay no graphs of their own and make no
 * host call that waits; rel_res is NaN as for any fixed-cycle solve.  Make one call outside the
 * capture first with the same shapes (it sets kernel attributes and, for the allocation-free
 * call, looks up the scratch array).  The other solves (batched, higher-order) return MG_EINVAL
 * under capture. */
#define MG_NO_GRAPH          0x4u  /* launch every kernel directly instead of replaying graphs    */
/* MG_NO_MEAN_FIX: f is taken as given, with no composite mean removed, and u is returned in the
 * gauge the iteration leaves it (no final zero-mean shift); stats.f_mean_removed is 0.  For a
 * caller whose f already has zero composite mean (tau from lpt2_source does): it saves the sum
 * and subtraction passes over f and the final pass over u.  The periodic problem needs that zero
 * mean (Section 3.2): with a nonzero mean the residual stalls at the mean's share of ||f|| and
 * the solve ends without converging (MG_ENOCONV at max_cycles, or MG_EDIVERGED once rounding
 * makes the stalled residual grow three cycles in a row).  Accepted by mg_solve_level, mg_solve_hierarchy, their
 * allocation-free variant and mg_solve_batch_hier; mg_solve_batch and the higher-order solves
 * reject it (MG_EINVAL). */
#define MG_NO_MEAN_FIX       0x8u

typedef struct {
    int n[3];       /* cells per axis (base: all three equal)                 */
    int off[3];     /* first covered parent cell (ignored for level 0)        */
    double h;       /* cell size; level p >= 1 must have h = h_{p-1} / 2       */
} mg_level;

typedef struct {
    int nlev;                       /* 1 + number of patches, 1..MG_MAX_LEVELS */
    mg_level lev[MG_MAX_LEVELS];
} mg_hier;

typedef struct {
    double tol;         /* stop when composite ||r|| / ||f|| <= tol (relative, after a cycle's step 9) */
    int max_cycles;     /* V-cycles at most (FP64 cycles, or FP32 inner cycles when mixed)            */
    int nu1, nu2;       /* pre / post red-black Gauss-Seidel sweeps (the paper uses 2 / 2)            */
    int prec;           /* MG_FP64 or MG_MIXED                                                        */
    unsigned flags;     /* MG_USE_INITIAL_GUESS | MG_FIXED_CYCLES | MG_NO_GRAPH | MG_NO_MEAN_FIX        */
    int inner;          /* mixed only: FP32 V-cycles per FP64 correction (1..16); 0 = chosen per      */
                        /* correction from the measured contraction, at most 4                      */
} mg_opts;

typedef struct {
    int cycles;                 /* V-cycles run (both precisions)                                */
    double rel_res;             /* final composite relative residual (NaN with MG_FIXED_CYCLES)   */
    double f_mean_removed;      /* composite mean subtracted from f                               */
    double res_hist[64];        /* res_hist[c-1]: relative residual after c cycles (first 64);   */
                                /* NaN where none was formed (mixed: one per `inner` cycles)      */
    long long cell_updates;     /* smoother cell-updates performed (all levels, both precisions)  */
} mg_stats;

/* ----------------------------------------------------------------------------------------------
 * Multigrid solves (Section 3.2 periodic FAS; Section 3.3 adaptive FAS on nested patches)
 * -------------------------------------------------------------------------------------------- */

/* Workspace bytes for mg_solve_level / mg_solve_hierarchy / mg_solve_batch member, exact. */
size_t mg_workspace_bytes(const mg_hier* hier, const mg_opts* opts);

/* Graph replay (mg_solve_level, mg_solve_hierarchy): the launch sequences a solve repeats - a
 * V-cycle with its residual norm, an outer step of the mixed-precision loop, the source
 * preparation and the final gauge - are captured as HIP graphs the second time one is met for a
 * workspace address and plan (shapes, spacings, sweep counts; for the preparation and gauge also
 * the f and u pointers) and replayed after that, with the same kernels in the same order, so the
 * same bits.  The graphs are cached per host thread for the life of the thread (at most 256); a
 * workspace freed and reused at the same address for the same plan replays them correctly.
 * Not used with MG_NO_GRAPH, with kernel timing on (mg_kprof_enable), or by the allocation-free
 * call. */

/* Periodic single level: solve L u = f - mean(f) on n^3 cells of size h.
 * n = 2^k * m with m in {1, 3, 5, 7} and n >= 2.  f (n^3 doubles) is read only.  u (n^3
 * doubles) receives the zero-mean solution; it is read only with MG_USE_INITIAL_GUESS.
 * stats may be NULL.  Errors: MG_EINVAL, MG_ENOCONV, MG_EDIVERGED, MG_EHIP. */
int mg_solve_level(int n, double h, const double* f, double* u, const mg_opts* opts,
                   mg_stats* stats, void* workspace, size_t workspace_bytes, void* stream);

/* Nested hierarchy: f[p], u[p] for p = 0..nlev-1, each with the level's cells.  Solves the
 * composite system (fine cells and uncovered coarse cells; covered coarse cells are the mean of
 * their 8 children) after removing the composite mean of f.  On return covered coarse cells of
 * u hold the mean of their children and the composite mean of u is zero. */
int mg_solve_hierarchy(const mg_hier* hier, const double* const* f, double* const* u,
                       const mg_opts* opts, mg_stats* stats, void* workspace,
                       size_t workspace_bytes, void* stream);

/* Allocation-free variant of mg_solve_hierarchy, for callers that cannot allocate: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same arguments,
 * operation, results (bit for bit) and errors as mg_solve_hierarchy, without the workspace: the
 * library's static device array of MG_SCRATCH_BYTES bytes serves as the workspace (one copy per
 * GPU, held until the process ends; the current device must be the stream's device).  Problems
 * whose mg_workspace_bytes exceed MG_SCRATCH_BYTES are rejected with MG_EINVAL (e.g. a 128^3
 * level fits in both precisions, 160^3 only in FP64).  The call makes no device, pinned-host or
 * event allocation: per-cycle residuals are read back into host stack memory, and kernel timing
 * (mg_kprof_enable) is ignored for its duration.  Every call on one GPU shares its array, which
 * keeps the last call's contents (nothing in it needs to start at zero): calls that overlap on
 * one GPU, from several host threads or streams, race and must be serialised by the caller. */
#define MG_SCRATCH_BYTES ((size_t)96 << 20)
int mg_solve_hierarchy_noalloc(const mg_hier* hier, const double* const* f, double* const* u,
                               const mg_opts* opts, mg_stats* stats, void* stream);

/* Periodic single level with the higher-order Laplacians of Table 1 (Section 3.2): the 1-D
 * stencil of order 2, 4 or 6 summed over the three axes (7, 13 or 19 points), on every level of
 * the same FAS V(nu1, nu2) cycle.  With a stencil wider than one cell, red-black is no longer a
 * 2-colouring; each half-sweep updates its colour from the values before it (Jacobi within the
 * colour), so the result does not depend on the update order.
 * n = 2^k with 2 <= n <= 1024 (coarsened to one cell); order = 2, 4 or 6; precision FP64
 * (opts->prec = MG_FP64), or mixed (MG_MIXED: FP32 V-cycles, opts->inner per FP64 correction, default 3,
 * inside FP64 defect correction with the same FP64 stopping test).  f and u: n^3 device doubles, [x][y][z], z
 * contiguous; f is read only; u receives the zero-mean solution of L u = f - mean(f) and is read
 * only with MG_USE_INITIAL_GUESS.  The solve iterates in u itself, which the kernels access as
 * 16-byte pairs of cells: u must be 16-byte aligned (MG_EINVAL otherwise).  stats and the stopping test as for mg_solve_level.
 * Workspace: mg_ho_workspace_bytes(n, order) bytes, 256-byte aligned (about 4.1 n^3 doubles,
 * the FP32 arrays of the mixed path included whatever the precision).
 * Errors: MG_EINVAL (size, order, h, options, workspace), MG_ENOCONV, MG_EDIVERGED, MG_EHIP. */
size_t mg_ho_workspace_bytes(int n, int order);   /* 0 for an invalid n or order */
int mg_solve_level_ho(int n, double h, int order, const double* f, double* u, const mg_opts* opts,
                      mg_stats* stats, void* workspace, size_t workspace_bytes, void* stream);

/* Nested hierarchy with the higher-order Laplacians of Table 1 (Section 3.3 with Tables 1 and 2):
 * the composite system of mg_solve_hierarchy with the operator of order 2, 4 or 6 on every level.
 * A patch reads R = order / 2 ghost layers on each face, refreshed before every half-sweep and
 * residual: a polynomial of degree `order` parallel to the face through the 2R + 1 parent cells
 * around the fine cell's parent (for each of the R parent layers outside the face), then one of
 * degree `order` normal to the face through those R values and the first R + 1 fine cells; the
 * ghosts of the 2 x 2 fine cells in front of one parent face are then shifted together so that the
 * mean of their fluxes (the Table 2 operator of order - 1) equals the parent's flux through that
 * face, whose covered cells are the means of their current children.  Half-sweeps update a colour
 * from the values before them (Jacobi within the colour), as in mg_solve_level_ho.
 * Arrays as in mg_solve_hierarchy (natural [x][y][z] order, one per level); the base n must be a
 * power of two (2..1024), patches at least `order` cells per axis, and the base must leave at
 * least order / 2 cells uncovered per axis.  FP64 only (opts->prec = MG_FP64).  On return covered
 * coarse cells of u hold the mean of their children and the composite mean of u is zero.
 * Workspace: mg_ho_hierarchy_workspace_bytes(hier, order) (0 for an invalid hierarchy or order).
 * Errors: MG_EINVAL, MG_ENOCONV, MG_EDIVERGED, MG_EHIP. */
size_t mg_ho_hierarchy_workspace_bytes(const mg_hier* hier, int order);
int mg_solve_hierarchy_ho(const mg_hier* hier, int order, const double* const* f, double* const* u,
                          const mg_opts* opts, mg_stats* stats, void* workspace, size_t workspace_bytes,
                          void* stream);

/* Composite residual r = f - L u of a hierarchy (covered coarse cells of r set to 0), with
 * f's composite mean removed first; u's covered coarse cells are first replaced by the mean of
 * their children (u is modified only there).  Writes sqrt(sum r^2 vol) / sqrt(sum f^2 vol)
 * to *rel (host pointer, may be NULL; synchronises the stream).  Workspace: mg_workspace_bytes. */
int mg_residual_hierarchy(const mg_hier* hier, const double* const* f, double* const* u,
                          double* const* r, double* rel, void* workspace,
                          size_t workspace_bytes, void* stream);

/* ----------------------------------------------------------------------------------------------
 * LPT (Section 3.1)
 * -------------------------------------------------------------------------------------------- */

/* Workspace bytes for lpt_displacements (what = 1), lpt2_source (what = 2) or lpt_lla_density
 * (what = 3), for either gradient order.  The LPT calls below need a base of at least 2^3 cells
 * (3^3 with the sixth-order gradient; MG_EINVAL otherwise). */
size_t lpt_workspace_bytes(const mg_hier* hier, int what);

/* psi_c = scale * G_c phi on every level, G the Table 1 gradient of order grad_order (4 or 6;
 * MG_EINVAL otherwise).  out[3*p + c] is the c-th component on level p.  The base wraps
 * periodically; patch cells next to a face use ghosts of width grad_order / 2 interpolated
 * tri-quadratically from the parent (covered parent cells taken as the mean of their children).
 * Covered coarse cells get the gradient of that mean.  phi is read only.  Asynchronous. */
int lpt_displacements(const mg_hier* hier, const double* const* phi, double* const* out,
                      int grad_order, double scale, void* workspace, size_t workspace_bytes,
                      void* stream);

/* tau[p] = sum_{i>j} (D_ii D_jj - D_ij^2) with D_ij = G_i G_j phi, G of order grad_order (4 or
 * 6), on every level (ghosts of width grad_order on patches), then covered coarse cells replaced
 * by the mean of their children and the composite mean removed, so tau is a compatible Poisson
 * source.  Asynchronous. */
int lpt2_source(const mg_hier* hier, const double* const* phi, double* const* tau, int grad_order,
                void* workspace, size_t workspace_bytes, void* stream);

/* Both of the above in one call (Section 3.1): out as lpt_displacements with this scale, tau as
 * lpt2_source, both with the gradient of order grad_order.  On the periodic base the second
 * derivatives are taken from out itself, D_ij = G_i out_j / scale, which saves one pass over the
 * base; with scale = +-1 tau is bit-identical to lpt2_source's, otherwise it differs by rounding.
 * scale must be finite and non-zero.  Workspace: lpt_workspace_bytes(hier, 2).  Asynchronous. */
int lpt_displacements_and_source(const mg_hier* hier, const double* const* phi, double* const* out,
                                 int grad_order, double scale, double* const* tau, void* workspace,
                                 size_t workspace_bytes, void* stream);

/* Baryon density of the local Lagrangian approximation (Section 5.3, eq. gasdens):
 *   delta[p] = rho / rho_bar - 1 = 1 / det(I + dL/dq) - 1,  (dL/dq)_ij = G4_j L_i,
 * at the Lagrangian cell centres of every level, for the displacement L = disp (+ disp2 when
 * disp2 is not NULL; e.g. the first- and second-order displacements of a 2LPT set).
 * disp[3*p + c] (and disp2[3*p + c]) is the c-th component on level p, natural [x][y][z] order,
 * as lpt_displacements writes it; delta[p] is one array per level and must not alias any
 * displacement array.  Inputs are read only.
 * On patches each component takes width-2 ghosts from its parent as in lpt_displacements (covered
 * parent cells as the mean of their children).  Then covered coarse cells of delta are replaced
 * by the mean of their children and the composite mean is subtracted from every level: the
 * paper's renormalisation that restores the mean density (mass conservation).  Cells past shell
 * crossing (det <= 0) are not detected: they give delta <= -1 or an infinity.
 * Workspace: lpt_workspace_bytes(hier, 3) (a few scalars for a single level; three copies of the
 * displacement and three padded patches for a hierarchy).  Asynchronous. */
int lpt_lla_density(const mg_hier* hier, const double* const* disp, const double* const* disp2,
                    double* const* delta, void* workspace, size_t workspace_bytes, void* stream);

/* ----------------------------------------------------------------------------------------------
 * Multi-scale Gaussian density on nested grids (Sections 2.1-2.3; sub-grid kernel mean of 3.5.3)
 *
 * delta = T * mu on every level of hier, with
 *   - T the real-space transfer function, given as radial[i] = T(i dr) (i < nradial, linear
 *     interpolation in r; the paper's FFTlog output), sampled on each level's displacement grid:
 *     the finest level directly or (subgrid != 0) as the mean over the 8 sub-cell centres at
 *     +-h/4; each coarser level as the mean over child pairs of the finer level's kernel (eq.
 *     transfer_average: fine displacements 2J-1, 2J, 2J+1 weighted 1/4, 1/2, 1/4 per axis) where
 *     the finer kernel grid reaches, T(|D|) elsewhere;
 *   - mu the white noise: xi[0] holds N^3 unit normals for the base, xi[p] (2 n_p)^3 unit normals
 *     on patch p's padded domain D'_p (twice the patch per axis, the patch centred at
 *     [n_p/2, 3 n_p/2)); level l's noise is xi / h_l^(3/2).  Each patch's noise keeps the modes of
 *     its parent below the parent's Nyquist (its coefficients replaced by 8 C(m) times the phase of
 *     the quarter-cell offset, C the DFT of the parent cells under D'), top down; then every
 *     covered parent cell's noise becomes the mean of its 8 children, finest first;
 *   - per patch: delta_self + delta_bnd (the noise inside the patch, and the noise minus its
 *     parent's value on the padding, convolved circularly on D') plus the conservative tri-cubic
 *     interpolation of the coarse contributions: the parent's noise outside the patch (the base:
 *     periodic; a parent patch: its own cells only) convolved with the parent's kernel, added to
 *     what the parent itself received.  delta_bnd's 8-child means are added to the parent's
 *     density on the parent cells under D' outside the patch.  Finally every covered coarse cell
 *     of delta is the mean of its children.
 * Geometry: a power-of-two cubic base (2..1024) and power-of-two patch sizes (4..512 per axis)
 * with the usual nesting (mg_workspace_bytes' rules); D'_p must lie inside the parent patch (the
 * base wraps; the first patch needs n <= N).  radial must reach every sampled radius (MG_EINVAL
 * names the radius otherwise).  xi and radial are read only; delta[l] is the level's own cells
 * (N^3, n_p^3).  All pointers are device memory; asynchronous on stream. */
size_t ic_density_workspace_bytes(const mg_hier* hier);
int ic_multiscale_density(const mg_hier* hier, const double* radial, int nradial, double dr,
                          int subgrid, const double* const* xi, double* const* delta,
                          void* workspace, size_t workspace_bytes, void* stream);

/* ----------------------------------------------------------------------------------------------
 * Spectral corrections that recover small-scale power (Section 3.5)
 *
 * Fields are real FP64 arrays of n[0] x n[1] x n[2] cells, natural [x][y][z] order, z contiguous,
 * device memory owned by the caller.  A periodic grid (isolated = 0) is transformed on its own
 * n points per axis (each n a power of two, 2..1024).  An isolated grid (isolated = 1: a patch,
 * with the field taken as zero outside it) is zero-padded at its origin corner to the smallest
 * power of two >= 2 n per axis (n <= 512), the paper's twice-the-size padding for power-of-two
 * patches; the padding is implicit (never stored).  Mode m of an axis of P points has wave number
 * k = 2 pi m / (P h), m in -P/2 .. P/2 - 1.
 * -------------------------------------------------------------------------------------------- */

#define SPEC_FV_DECONV 1   /* Section 3.5.1: divide by prod_i sinc(k_i h / 2), the cell average */
#define SPEC_SG_DECONV 2   /* Section 3.5.3: divide by prod_i cos(k_i h / 4), the 8-sub-cell mean */

/* Workspace bytes of spec_deconvolve and lpt_hybrid_correction for this shape (0 if invalid). */
size_t spec_workspace_bytes(const int n[3], int isolated);

/* out = the deconvolution of f (kind SPEC_FV_DECONV or SPEC_SG_DECONV): f's transform divided by
 * the window's transform, back-transformed.  The mean (k = 0) is unchanged.  out may alias f.
 * MG_EINVAL for an unknown kind, a NULL pointer, a shape outside the limits above or a workspace
 * that is too small or not 256-byte aligned.  Asynchronous on stream. */
int spec_deconvolve(const int n[3], int kind, int isolated, const double* f, double* out,
                    void* workspace, size_t workspace_bytes, void* stream);

/* The exact discrete periodic Poisson solve by eigenvalue division (Section 3.2 with Table 1's
 * symbols): u~ = f~ / lambda(k), lambda the symbol of the order-2, 4 or 6 Laplacian summed over
 * the axes, the k = 0 mode zero (the zero-mean solution of L u = f - mean f).  This is the fixed
 * point the periodic multigrid solves converge to; the bench measures their error against it.
 * Periodic only (n[a] powers of two, 2..1024); workspace spec_workspace_bytes(n, 0); u may alias
 * f.  Asynchronous on stream. */
int spec_poisson(const int n[3], double h, int order, const double* f, double* u,
                 void* workspace, size_t workspace_bytes, void* stream);

/* Hybrid Poisson solver (Section 3.5.2): ADDS to out3[c] (c = x, y, z) the correction that turns
 * the finite-difference displacement scale * G_c phi, L phi = f (L the Table 1 Laplacian of
 * lap_order 2, 4 or 6, G the gradient of grad_order 4 or 6), into the k-space exact
 * scale * d_c (laplacian^-1 f):
 *   out3[c] += IFFT( i scale [ -k_c / k^2 - g_c / lambda ] h FFT(f) ),
 * g_c and lambda the gradient and Laplacian symbols in grid units.  k = 0 and the Nyquist plane
 * of axis c get no correction.  On the periodic base of a single-level setup this makes the
 * result a pure FFT Poisson solve; on the finest patch (isolated = 1) f is zero outside the patch.
 * f is read only and must not alias an output.  Asynchronous on stream. */
int lpt_hybrid_correction(const int n[3], double h, int isolated, int lap_order, int grad_order,
                          double scale, const double* f, double* const* out3, void* workspace,
                          size_t workspace_bytes, void* stream);

/* ----------------------------------------------------------------------------------------------
 * Batched independent periodic solves (many small instances in one persistent launch)
 * -------------------------------------------------------------------------------------------- */

/* Workspace bytes for a batch of ninst periodic instances of sizes n[i] (exact; independent of
 * the spacings). */
size_t mg_batch_workspace_bytes(int ninst, const int* n, const mg_opts* opts);

/* Solve ninst independent periodic problems (sizes n[i], spacings h[i], device pointers f[i],
 * u[i]; the pointer arrays themselves are host arrays).  Each instance's result, cycle count and
 * residual history are bit-identical to mg_solve_level with the same options; stats (host array
 * of ninst, may be NULL) per instance.  Instances with even n and n^3 > 16^3 share batched
 * launches: one launch per V-cycle step and level depth for all of them, and one launch that
 * runs the small-level tails of all of them (one workgroup each).  These launch sequences are
 * captured as HIP graphs on first use for a workspace and batch shape and replayed every cycle
 * (MG_NO_GRAPH: launched directly); converged instances are switched off by a device flag.
 * Other instances are solved one by one in the same call.  The smoother's block size and cells
 * per thread are chosen per level depth by timing candidates once per batch shape and process.
 * Synchronises the stream at least once per FP64 correction (mixed) or cycle (FP64).
 * Returns the first failure in instance order (MG_ENOCONV / MG_EDIVERGED; all instances are
 * still solved and their stats filled), or MG_EINVAL / MG_EHIP. */
int mg_solve_batch(int ninst, const int* n, const double* h, const double* const* f,
                   double* const* u, const mg_opts* opts, mg_stats* stats, void* workspace,
                   size_t workspace_bytes, void* stream);

/* Workspace bytes for mg_solve_batch_hier over these instances (exact; 0 with the reason in
 * mg_last_error when an instance or the options are invalid). */
size_t mg_batch_hier_workspace_bytes(int ninst, const mg_hier* const* hier, const mg_opts* opts);

/* Solve ninst independent problems, each a hierarchy (Sections 3.2-3.3: a periodic base with
 * 0..7 nested patches).  hier[i] describes instance i; f[i][p], u[i][p] are the device arrays of
 * its level p (the pointer arrays are host arrays); stats (host array of ninst, may be NULL) per
 * instance.  Each instance's result, cycle count and residual history are bit-identical to
 * mg_solve_hierarchy with the same options.  Single-level instances share the batched launches
 * of mg_solve_batch on `stream` (with MG_NO_MEAN_FIX they are solved like the others); the
 * instances with patches run concurrently, up to three at a time, largest first, each as its own solve on a library-owned stream of default priority
 * driven by a library worker thread (created on first use, kept until the process ends).  Those
 * streams start after the work already queued on `stream`, and later work on `stream` waits for
 * them.  Calls are serialised: one hierarchy batch at a time per process.  Returns MG_EINVAL
 * (arguments, before any device work) or MG_EHIP if any part failed, else the first instance, in
 * instance order, that did not converge (MG_ENOCONV) or diverged (MG_EDIVERGED); all instances
 * are still solved and their stats filled. */
int mg_solve_batch_hier(int ninst, const mg_hier* const* hier, const double* const* const* f,
                        double* const* const* u, const mg_opts* opts, mg_stats* stats, void* workspace,
                        size_t workspace_bytes, void* stream);

/* Autotuning of the batched smoother (block size and cells per thread, per level depth).
 * mg_batch_tune_candidates: the number of candidate shapes.  mg_batch_force_shape(i): every
 * later mg_solve_batch in the process uses candidate i at every depth without timing (i = -1:
 * back to timing; MG_EINVAL out of range); every candidate gives the same bits.
 * mg_tune_cache(path): the tuned shapes persist in a JSON file at path - entries already in it
 * are loaded (the return value is their number; MG_EINVAL if the file is not a tuning cache), and
 * every new tuning rewrites it; NULL or "" stops the persistence (returns 0).  Process-wide. */
int mg_batch_tune_candidates(void);
int mg_batch_force_shape(int index);
int mg_tune_cache(const char* path);

/* Autotuning of the mixed-precision solo solve's FP32 inner cycles per FP64 correction: solves
 * hier (f -> u, zero start) with every count 0..4 (0: the contraction rule of the default), each
 * twice after a graph-capturing first call, timed with events on stream; *best gets the fastest
 * count and ms[k] (5 entries, or NULL) each count's time in ms (-1 where the solve failed).  The
 * choice is recorded for the problem's shape (level sizes and offsets, nu1, nu2 and the decade of
 * tol) and persists through mg_tune_cache; from then on every mixed mg_solve_level /
 * mg_solve_hierarchy / mg_solve_hierarchy_noalloc of that shape with opts->inner = 0 uses it.
 * u is left holding the last candidate's solution.  MG_EINVAL for an FP64 opts or a bad
 * hierarchy; the last solve error if no count converged.  Synchronises the stream. */
int mg_tune_inner(const mg_hier* hier, const double* const* f, double* const* u,
                  const mg_opts* opts, int* best, double* ms, void* workspace,
                  size_t workspace_bytes, void* stream);

/* ----------------------------------------------------------------------------------------------
 * Single steps, exposed for kernel-level parity checks
 * -------------------------------------------------------------------------------------------- */

/* `half_sweeps` red/black half-sweeps (red first) of Section 3.2's smoother on a periodic n^3
 * level in place: u <- (sum of 6 neighbours - h^2 f) / 6 on one colour.  prec = MG_FP64 works
 * on u and f directly; MG_MIXED rounds u and f to float32, sweeps in float32 and widens back.
 * Workspace: mg_workspace_bytes of the single level. */
int mg_smooth_level(int n, double h, const double* f, double* u, int half_sweeps, int prec,
                    void* workspace, size_t workspace_bytes, void* stream);

/* Flux-matched ghost layer of patch p (Section 3.3) from u[p-1] and u[p].  ghosts receives the
 * 6 faces back to back: x-low, x-high ([ny][nz] each), y-low, y-high ([nx][nz]), z-low,
 * z-high ([nx][ny]).  flux_match = 0 gives the interpolated guess without flux matching. */
int mg_ghost_fill(const mg_hier* hier, int p, const double* const* u, double* ghosts,
                  int flux_match, void* stream);

/* The R = order / 2 ghost layers of patch p for the operator of this order (Section 3.3, Tables 1
 * and 2; the construction of mg_solve_hierarchy_ho) from u[p-1] and u[p] (natural order, as the
 * caller holds them).  ghosts receives the 6 faces back to back: x-low, x-high ([R][ny][nz] each,
 * layer 0 next to the face), y-low, y-high ([R][nx][nz]), z-low, z-high ([R][nx][ny]).
 * flux_match = 0 gives the interpolated values without the flux shift. */
int mg_ghost_fill_ho(const mg_hier* hier, int order, int p, const double* const* u, double* ghosts,
                     int flux_match, void* stream);

/* ----------------------------------------------------------------------------------------------
 * Measurement support
 * -------------------------------------------------------------------------------------------- */

/* period > 0 (per calling thread): every period-th launch of the smoother on the finest level of
 * a solve (the first, then every period-th after it) is stamped by two HIP events recorded by the
 * dispatch itself on the launch stream; 1 times every launch, 0 switches timing off.  Each timed
 * launch costs several microseconds of extra dispatch work, so a period above 1 keeps that out
 * of the work being timed.  Negative periods are rejected (MG_EINVAL). */
int mg_kprof_enable(int period);

/* Wait for the recorded events, return the summed launch durations (ms), the number of timed
 * launches and their algorithmic bytes (3 words per cell-update: u in, f in, u out), and reset. */
int mg_kprof_read(double* ms_total, long long* launches, double* bytes_total);

const char* mg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MGIC_H */
