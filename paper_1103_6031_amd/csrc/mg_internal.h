// Internal declarations shared by the HIP kernel translation units and the host solver.
// Not part of the public ABI (see include/mgic.h).
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

#include "fastdiv.h"

namespace mgic {

constexpr int kBlock = 256;          // threads per workgroup (4 wave64)
constexpr int kMaxPartials = 4096;   // partial sums per reduction (fixed => deterministic)
constexpr int kRedV = 4;             // cells per thread per pass in the reduction kernels

// A 3-D box of cells.
struct Dims {
    int x, y, z;
    __host__ __device__ size_t cells() const { return (size_t)x * y * z; }
};

// Storage of one level: natural rows, or the colour-split rows of periodic levels (each row of
// z holds its red cells, (x+y+z) even, in increasing z, then its black cells).
// The dividers are always derived from d by the constructor, so a Lay can never decode with
// stale constants; device code that only needs indices uses (Dims, split) directly.
__host__ __device__ inline int log2_exact(int n) {   // log2 n if n is a power of two, else -1
    if (n < 1 || (n & (n - 1))) return -1;
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

struct Lay {
    Dims d{1, 1, 1};
    int split = 0;
    FastDiv dz, dy, dzh;   // division by d.z, d.y and d.z / 2
    int lgx = -1, lgy = -1, lgz = -1;   // log2 of the dims (-1: not a power of two)
    int pow2 = 0;                       // all three dims are powers of two and d.z >= 2

    Lay() = default;
    __host__ __device__ Lay(Dims d_, int split_)
        : d(d_), split(split_), dz((unsigned)d_.z), dy((unsigned)d_.y),
          dzh((unsigned)(d_.z > 1 ? d_.z / 2 : 1)), lgx(log2_exact(d_.x)), lgy(log2_exact(d_.y)),
          lgz(log2_exact(d_.z)) {
        pow2 = lgx >= 0 && lgy >= 0 && lgz >= 1;
    }
};
inline Lay mklay(Dims d, int split) { return Lay(d, split); }

// storage position of cell (x, y, z)
__host__ __device__ __forceinline__ size_t lidx(Dims d, int split, int x, int y, int z) {
    const size_t row = (size_t)x * d.y + y;
    if (!split) return row * d.z + z;
    return row * d.z + (((x + y + z) & 1) ? (size_t)(d.z >> 1) : 0) + (z >> 1);
}
__host__ __device__ __forceinline__ size_t lidx(const Lay& L, int x, int y, int z) {
    if (L.pow2) {   // shifts instead of multiplies (every level fits in 2^31 cells)
        const unsigned row = ((unsigned)x << L.lgy) | (unsigned)y;
        if (!L.split) return (size_t)((row << L.lgz) | (unsigned)z);
        return (size_t)((row << L.lgz) + (((x + y + z) & 1) ? (1u << (L.lgz - 1)) : 0u) + ((unsigned)z >> 1));
    }
    return lidx(L.d, L.split, x, y, z);
}

// coordinates of storage position i (every level has fewer than 2^31 cells)
__host__ __device__ __forceinline__ void ldecode(const Lay& L, size_t i64, int& x, int& y, int& z) {
    const unsigned i = (unsigned)i64;
    unsigned row;
    int p;
    if (L.pow2) {
        row = i >> L.lgz;
        p = (int)(i & ((1u << L.lgz) - 1));
        x = (int)(row >> L.lgy);
        y = (int)(row & ((1u << L.lgy) - 1));
    } else {
        row = L.dz.div(i);
        p = (int)(i - row * (unsigned)L.d.z);
        const unsigned xq = L.dy.div(row);
        y = (int)(row - xq * (unsigned)L.d.y);
        x = (int)xq;
    }
    if (!L.split) {
        z = p;
        return;
    }
    const int nzh = L.d.z >> 1;
    const int col = p >= nzh;
    z = 2 * (p - col * nzh) + ((x + y + col) & 1);
}

// Block numbering of the grid kernels.  Workgroups go round-robin over the 8 XCDs; measured on
// MI355X, renumbering them so that each XCD sweeps one contiguous eighth of a level (to keep
// neighbour rows in one L2) was slower for every stencil here (e.g. the FP64 half-sweep at 256^3
// by 9%), so blocks keep the dispatch order.
__device__ __forceinline__ size_t xcd_block() { return blockIdx.x; }
__device__ __forceinline__ size_t lpt_block() { return blockIdx.x; }

// Where a fine level's coarse representation lives inside its parent array.  Built only by the
// constructor from the parent's layout, so its dims, storage and fast-index data agree.
struct ParentMap {
    Lay pl;             // parent array: dims, storage (natural or colour-split), index data
    int off[3] = {0, 0, 0};   // first covered parent cell
    int periodic = 0;   // parent is periodic (base or a coarsening of it)

    ParentMap() = default;
    __host__ __device__ ParentMap(const Lay& parent, int o0, int o1, int o2, int per)
        : pl(parent), off{o0, o1, o2}, periodic(per) {}
};


// Covered box of a level (cells owned by the next finer level); n = 0 means none.
struct CovBox {
    int lo[3];
    int n[3];
};

// Face layout of a patch ghost array: x-lo, x-hi [ny][nz]; y-lo, y-hi [nx][nz]; z-lo, z-hi [nx][ny].
__host__ __device__ inline size_t ghost_face_offset(Dims d, int face) {
    const size_t fx = (size_t)d.y * d.z, fy = (size_t)d.x * d.z, fz = (size_t)d.x * d.y;
    switch (face) {
        case 0: return 0;
        case 1: return fx;
        case 2: return 2 * fx;
        case 3: return 2 * fx + fy;
        case 4: return 2 * fx + 2 * fy;
        case 5: return 2 * fx + 2 * fy + fz;
        default: return 2 * fx + 2 * fy + 2 * fz;  // face 6: total size of the 6 faces
    }
}
__host__ __device__ inline size_t ghost_cells(Dims d) { return ghost_face_offset(d, 6); }

// One periodic level of the single-workgroup tail V-cycle (lev[0] finest, lev[n-1] coarsest).
constexpr int kTailThreads = 1024;
constexpr size_t kTailMaxCells = 16 * 16 * 16;   // levels at or below this size join the tail
constexpr size_t kTailMaxLds = 160 * 1024;        // LDS one gfx950 workgroup may hold
constexpr size_t kTailLdsBound = 96 * 1024;       // dynamic LDS any tail plan needs (levels <= 16^3)
constexpr int kTailMaxLevels = 8;
template <class T>
struct TailLevel {
    T* u;       // the level's global arrays (only level 0's are read and written)
    T* f;
    Lay lay;    // colour-split except the odd (or single-cell) coarsest level
    double h;
    unsigned lds_u, lds_f, lds_o;   // byte offsets in LDS of u, f and the restricted copy (uold)
};
template <class T>
struct TailPlan {
    int n, nu1, nu2;
    int inst;                       // batched launches: the instance (index of its active flag)
    int fas0;                       // 1: level 0's f still lacks the FAS term L u (step 6), add it first
    unsigned lds_bytes;             // total LDS, including the coarsest solver's 2 x 343 doubles
    TailLevel<T> lev[kTailMaxLevels];
};
// Places every tail level in LDS (u, f, then the copy of the restricted u of the next level),
// 16-byte aligned; the coarsest solver's tables follow.  Offsets live in the plan so that the
// kernel forms its pointers with scalar arithmetic instead of indexing a private array.
template <class T>
inline unsigned tail_assign_lds(TailPlan<T>& tp) {
    size_t off = 0;
    for (int k = 0; k < tp.n; ++k) {
        const size_t c = tp.lev[k].lay.d.cells();
        tp.lev[k].lds_u = (unsigned)off;
        off += c * sizeof(T);
        tp.lev[k].lds_f = (unsigned)off;
        off += c * sizeof(T);
        tp.lev[k].lds_o = (unsigned)off;
        if (k + 1 < tp.n) off += (c / 8) * sizeof(T);
        off = (off + 15) & ~(size_t)15;
    }
    tp.lds_bytes = (unsigned)(off + 2 * 343 * sizeof(double));
    return tp.lds_bytes;
}

// Segments of partial sums combined by the finalize kernel: out = sum_s w[s] * sum(partials[s]).
struct SegList {
    int n;
    int off[16];
    int cnt[16];
    double w[16];
};

// ----------------------------------------------------------------------------------------------
// launchers (defined in the .hip files); all enqueue on `st`
// ----------------------------------------------------------------------------------------------
template <class T> void launch_fill(T* p, size_t n, T v, hipStream_t st);
template <class A, class B> void launch_relayout(const A* src, Lay ls, B* dst, Lay ld, hipStream_t st);
void launch_add_f32_to_f64(double* u, const float* e, size_t n, hipStream_t st);
template <class T> void launch_sub_mean(T* a, size_t n, const double* sum, double inv_count, hipStream_t st);

// red-black half-sweep (colour 0 = red = (x+y+z) even); ghosts == nullptr => periodic level in
// the colour-split layout, else a patch in natural rows with its ghost faces
// ev0 / ev1 (both null, or both events): stamped by the dispatch itself at the kernel's start and
// end, so their elapsed time is the kernel's own duration
template <class T> void launch_rbgs_half(T* u, const T* f, const T* ghosts, Lay L, double h,
                                         int colour, hipStream_t st, hipEvent_t ev0 = nullptr,
                                         hipEvent_t ev1 = nullptr);

// residual r = f - L u on the fine level, restricted: parent u[cov] = mean8 u, uold = mean8 u,
// parent f[cov] = mean8 r  (fine level periodic if ghosts == nullptr)
template <class T> void launch_resid_restrict(const T* u, const T* f, const T* ghosts, Lay L, double h,
                                              T* pu, T* pf, T* uold, ParentMap pm, hipStream_t st);
// parent f[cov] += L u  (FAS coarse right-hand side), L over the parent's own stencil
template <class T> void launch_fas_rhs(const T* pu, T* pf, ParentMap pm, Dims cov, double H, hipStream_t st);
// fine u += inject(parent u[cov] - uold); black_only on a colour-split level corrects the black
// cells only (valid when a red half-sweep follows: it rewrites every red cell unread)
template <class T> void launch_prolong(T* u, Lay L, const T* pu, const T* uold, ParentMap pm, int black_only,
                                       hipStream_t st);
// V-cycle over all levels of a tail plan in one single-workgroup launch
template <class T> void launch_tail(const TailPlan<T>& tp, hipStream_t st);
// fused pre / post legs of a periodic power-of-two coarsening of edge n (16, 32 or 64), one workgroup
// per 8^3 tile (bit-identical to the one-step kernels)
bool level_fusable(int n, int nu1, int nu2);
// steps 3-5, 8 (black cells) and 6 on periodic colour-split power-of-two cubes of edge n (the
// coarse level of edge n / 2 for the first two), with the arithmetic of the generic kernels
template <class T>
void launch_resid_restrict_p2(const T* u, const T* f, int n, double h, T* pu, T* pf, T* uold, hipStream_t st);
template <class T> void launch_prolong_black_p2(T* u, int n, const T* pu, const T* uold, hipStream_t st);
template <class T> void launch_fas_rhs_p2(const T* pu, T* pf, int n, double H, hipStream_t st);
// red-black half-sweep with 16-byte accesses on a periodic colour-split power-of-two level whose
// half-rows hold a multiple of 16 bytes (rbgs_vec_ok); same bits as launch_rbgs_half
bool rbgs_vec_ok(const Lay& L, size_t elem);
// step 8 on the black cells and the first red half-sweep of step 9 in one pass (the corrected
// black values are read, not stored: the black half-sweep after it rewrites them); pu is the
// coarse level's u, uold this level's restricted copy; periodic power-of-two cube, rbgs_vec_ok
// step 6 on a whole periodic colour-split power-of-two cube of edge n with 16-byte runs (both
// colours of a run per thread; half-rows a multiple of 16 bytes); same bits as launch_fas_rhs_p2
template <class T> void launch_fas_vec(const T* pu, T* pf, int n, double H, hipStream_t st);
template <class T>
void launch_rbgs_vec_corr(T* u, const T* f, const Lay& L, double h, const T* pu, const T* uold, hipStream_t st);
template <class T>
void launch_rbgs_vec(T* u, const T* f, const Lay& L, double h, int colour, hipStream_t st, hipEvent_t ev0,
                     hipEvent_t ev1);
template <class T>
void launch_level_pre(const T* u, const T* f, T* uo, T* fo, T* pu, T* pf, T* uold, int n, double h, int nu1,
                      hipStream_t st);
template <class T>
void launch_level_post(const T* ui, const T* fi, const T* uc, const T* uold, T* uout, int n, double h, int nu2,
                       hipStream_t st);
// exact coarsest solve on an odd periodic M^3 grid (M = 1: u = 0)
template <class T> void launch_coarsest(T* u, const T* f, int M, double h, hipStream_t st);

// flux-matched ghost layer of a patch (arithmetic in double, stored as T).  part (2 doubles per
// ghost cell, or null) holds the parent's part of each value between the fills of one smoothing
// pass: mode 1 computes and stores it, mode 2 reuses it (valid while the parent is unchanged and
// the last mode-1 fill used the same parent array), mode 0 neither.
template <class T> void launch_ghost_fill(const T* pu, const T* u, T* ghosts, Lay L, ParentMap pm,
                                          int flux_match, hipStream_t st, double* part = nullptr,
                                          int mode = 0);
// parent[cov] = mean8(fine)
template <class T> void launch_restrict_cov(const T* fine, Lay L, T* parent, ParentMap pm, hipStream_t st);

// residual of one level: per-block partial sums of r^2 over cells outside `cov`; r written to
// rout (if non-null; cells inside cov get 0)
template <class T, class R> void launch_residual(const T* u, const T* f, const T* ghosts, Lay L, double h,
                                                 CovBox cov, R* rout, Lay LR, double* partials, int* nparts,
                                                 hipStream_t st);
// fused outer step of the mixed-precision defect correction on a colour-split periodic level:
// u_out = u_in + e_in, rhs = (float)(f - L u_out), red e_out = first red half-sweep from e = 0;
// per-block partial sums of r^2.  u_in == nullptr: u_in taken as +0 (not read); if e_in is null
// as well (the first step of a zero start), u_out is not written either - the caller keeps the
// zero iterate implicit and passes u_in == nullptr again with the next correction
void launch_outer_split(const double* u_in, const float* e_in, const double* f, double* u_out, float* rhs,
                        float* e_out, Lay L, double h, double* partials, int* nparts, hipStream_t st);
// per-block partial sums of a (or a^2) over cells outside cov
void launch_sum(const double* a, Lay L, CovBox cov, int square, double* partials, int* nparts, hipStream_t st);
void launch_finalize(const double* partials, SegList segs, double* out, hipStream_t st);
// fused passes (partials as launch_sum over the level array): dst (layout L) = src (natural) with
// the sum of the values; a -= sum * inv with the sum of squares; dst (ld) = src (ls) - sum * inv
void launch_relayout_sum(const double* src, double* dst, Lay L, double* partials, int* nparts, hipStream_t st);
void launch_submean_sumsq(double* a, Lay L, const double* sum, double inv, double* partials, int* nparts,
                          hipStream_t st);
void launch_relayout_sub(const double* src, Lay ls, double* dst, Lay ld, const double* sum, double inv,
                         hipStream_t st);

// LPT: padded copy with tri-quadratic ghosts of width R from the parent (covered parent cells
// must already hold the mean of their children)
void launch_wide_ghost(const double* pu, const double* u, double* padded, Dims d, ParentMap pm, int R,
                       hipStream_t st);
// psi_c = scale * G_c phi with the Table 1 gradient of `order` (4 or 6); src is periodic (R = 0)
// or padded by R >= order / 2
void launch_grad4(const double* src, int R, Dims d, double h, double scale, double* ox, double* oy,
                  double* oz, hipStream_t st, int order = 4);
// tau = sum_{i>j} D_ii D_jj - D_ij^2, D = G o G of `order`; src periodic (R = 0) or padded by
// R >= order; psi is scratch for 3 arrays of (d + 2(R - order/2))^3 (d^3 when periodic)
void launch_tau(const double* src, int R, Dims d, double h, double* tau, double* psi, hipStream_t st,
                int order = 4);
// tau on a periodic level from the three components g_c = s G_c phi of a scaled gradient
// (post = 1 / s^2)
void launch_tau_from_grad(const double* g0, const double* g1, const double* g2, Dims d, double h, double post,
                          double* tau, hipStream_t st, int order = 4);
// LLA overdensity 1 / det(I + G4 L) - 1 with L = a (+ b when b is given), three components each,
// periodic (R = 0) or padded by R >= 2
void launch_lla(const double* const* a, const double* const* b, int R, Dims d, double h, double* out, hipStream_t st);
// dst = a + b elementwise
void launch_add2(const double* a, const double* b, double* dst, size_t n, hipStream_t st);

// ----------------------------------------------------------------------------------------------
// batched launches: many independent periodic instances in one grid
// ----------------------------------------------------------------------------------------------
// One instance's share of a batched launch: blocks [blk0, blk0 + nblk) of the grid do exactly
// what a plain launch of nblk blocks does on that instance alone (same cells per block, same
// reduction striding), so every instance gets the bits of its own solo solve.
struct BSeg {
    int inst;           // instance: index of its active flag
    unsigned blk0;      // first block of the segment
    unsigned nblk;      // blocks of the segment
    Lay L;              // the instance's level
    Lay C;              // transfers: the covered coarse box, natural order; relayout: destination
    ParentMap pm;       // transfers: the coarse representation inside the parent
    double h;           // level spacing (FAS right-hand side: the parent's; mean removal: 1/cells)
    void* a[6];         // arrays, listed per batched kernel
    double* part;       // reductions: nblk partial sums of this instance
};
// per-instance finalize of a batched reduction: *out = w * sum(part[0..cnt)), one block each
struct BFin {
    const double* part;
    int cnt;
    double w;
    double* out;
};

inline int grid_for(size_t n, int per_block = kBlock, int cap = 1 << 30) {
    size_t g = (n + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > (size_t)cap) g = cap;
    return (int)g;
}

// batched launchers; `active` (device, one int per instance) skips finished instances.
// rbgs: a = {u, f}, colour as given; block threads, V cells per thread
template <class T> void launch_b_rbgs(const BSeg* segs, int nseg, unsigned grid, int block, int V, const int* active,
                                      int colour, hipStream_t st);
// a = {u, f, pu, pf, uold}: residual + restriction (steps 3-5)
template <class T> void launch_b_resid_restrict(const BSeg* segs, int nseg, unsigned grid, const int* active,
                                                hipStream_t st);
// a = {pu, pf}: FAS right-hand side (step 6), h = the parent's spacing
template <class T> void launch_b_fas(const BSeg* segs, int nseg, unsigned grid, const int* active, hipStream_t st);
// a = {u, pu, uold}: step 8 (black cells only if black_only)
template <class T> void launch_b_prolong(const BSeg* segs, int nseg, unsigned grid, const int* active,
                                         int black_only, hipStream_t st);
// sets the batched kernels' function attributes (LDS size); call before any graph capture
hipError_t batch_kernel_setup();
hipError_t tail_kernel_setup();
// the single-workgroup tails of n instances, one workgroup each
template <class T> void launch_b_tail(const TailPlan<T>* plans, int n, unsigned lds_bytes, const int* active,
                                      hipStream_t st);
// a = {u_in, e_in, f, u_out, rhs, e_out}: fused mixed-precision outer step (e_in unused if !has_e;
// zero_u: u_in is taken as zero and not read)
void launch_b_outer(const BSeg* segs, int nseg, unsigned grid, const int* active, int has_e, int zero_u,
                    hipStream_t st);
// a = {u, f}: FP64 residual partial sums
void launch_b_residual(const BSeg* segs, int nseg, unsigned grid, const int* active, hipStream_t st);
// a = {v}: partial sums of v (square: of v^2)
void launch_b_sum(const BSeg* segs, int nseg, unsigned grid, const int* active, int square, hipStream_t st);
void launch_b_finalize(const BFin* fins, int n, const int* active, hipStream_t st);
// a = {v, sum}: v -= sum * h  (h holds 1 / cells)
void launch_b_sub_mean(const BSeg* segs, int nseg, unsigned grid, const int* active, hipStream_t st);
// a = {src, dst}: dst (layout C) = src (layout L)
void launch_b_relayout(const BSeg* segs, int nseg, unsigned grid, const int* active, hipStream_t st);
// the fused passes of launch_relayout_sum / launch_submean_sumsq / launch_relayout_sub per segment:
// a = {src natural, dst}; a = {array, sum} with h = 1 / cells; a = {src, dst, sum} with h = 1 / cells
void launch_b_relayout_sum(const BSeg* segs, int nseg, unsigned grid, const int* active, hipStream_t st);
void launch_b_submean_sumsq(const BSeg* segs, int nseg, unsigned grid, const int* active, hipStream_t st);
void launch_b_relayout_sub(const BSeg* segs, int nseg, unsigned grid, const int* active, hipStream_t st);
// a = {p}: p = 0 over L's cells
template <class T> void launch_b_zero(const BSeg* segs, int nseg, unsigned grid, const int* active, hipStream_t st);

// periodic FAS with the order-2/4/6 Laplacians of Table 1 (k_highorder.hip): n = 2^lg per axis,
// natural order, FP64.  The half-sweep is out of place (reads in, writes every cell of out).
constexpr int kHoParts = 8192;   // partial sums of the reductions, at most
template <class T>
void launch_ho_half(const T* in, T* out, const T* f, int lg, double h, int order, int colour, hipStream_t st,
                    hipEvent_t ea = nullptr, hipEvent_t eb = nullptr);
template <class T>   // h: the fine spacing
void launch_ho_resid_restrict(const T* u, const T* f, T* uc, T* uold, T* rc, int lgc, double h, int order,
                              hipStream_t st);
template <class T> void launch_ho_fas(const T* uc, T* fc, int lgc, double hc, int order, hipStream_t st);
template <class T> void launch_ho_prolong(T* u, const T* uc, const T* uold, int lg, hipStream_t st);
template <class T> void launch_ho_fill(T* a, int lg, T v, hipStream_t st);
// mixed precision: r32 = f - L u (FP64) with out[0] = sum r^2; u += e32
void launch_ho_resid32(const double* u, const double* f, float* r32, int lg, double h, int order, double* part,
                       double* out, hipStream_t st);
void launch_ho_add32(double* u, const float* e, int lg, hipStream_t st);
void launch_ho_sum(const double* a, int lg, double* part, double* out, hipStream_t st);
void launch_ho_sub(const double* a, const double* sum, double* out, int lg, double* part, double* sumsq,
                   hipStream_t st);
void launch_ho_rnorm(const double* u, const double* f, int lg, double h, int order, double* part, double* out,
                     hipStream_t st);

// ----------------------------------------------------------------------------------------------
// higher-order Laplacians on nested patches (k_highorder.hip): natural order, FP64.  A patch of
// radius-R operator keeps R ghost layers per face: x-low, x-high [R][ny][nz], y-low, y-high
// [R][nx][nz], z-low, z-high [R][nx][ny], layer 0 next to the face.
// ----------------------------------------------------------------------------------------------
struct HozPatch {
    int n[3];      // cells per axis (even)
    int off[3];    // first covered parent cell
    int pn[3];     // parent dims
    int pper;      // the parent is the periodic base
    double h;      // spacing (the parent's is 2h)
};
// ghost-zone weights for radius R: Lagrange weights of the parallel step (nodes -R..R, at child
// offsets -1/4 and +1/4), of the normal step for each ghost layer (R coarse nodes, then R + 1 fine
// ones) and the Table 2 flux operator with the sum of its R ghost-side weights
struct HozW {
    double par[2][7];
    double nor[3][7];
    double F[6];
    double S;
};
__host__ __device__ inline size_t hoz_face_off(const int* n, int R, int face) {
    const size_t fx = (size_t)R * n[1] * n[2], fy = (size_t)R * n[0] * n[2], fz = (size_t)R * n[0] * n[1];
    const size_t o[7] = {0, fx, 2 * fx, 2 * fx + fy, 2 * fx + 2 * fy, 2 * fx + 2 * fy + fz, 2 * fx + 2 * fy + 2 * fz};
    return o[face];
}
// ghost layers of a patch; part (2R doubles per face column, hoz_face_off(n, 1, 6) columns, or
// null) holds the parent's part of the values between the fills of one smoothing pass: mode 1
// computes and stores it, mode 2 reuses it (parent unchanged since the last mode-1 fill), mode 0
// neither
void launch_hoz_ghost(const double* pu, const double* u, double* g, const HozPatch& P, const HozW& W, int order,
                      int flux_match, hipStream_t st, double* part = nullptr, int mode = 0);
void launch_hoz_half(const double* in, double* out, const double* f, const double* g, const HozPatch& P, int order,
                     int colour, hipStream_t st);
// steps 3-5: parent u and f on the covered cells := the means of the children's u and residual,
// uold := the same mean of u
void launch_hoz_resid_restrict(const double* u, const double* f, const double* g, const HozPatch& P, int order,
                               double* pu, double* pf, double* uold, hipStream_t st);
// step 6 on the covered box of a level: f += L u (periodic power-of-two base, or a patch whose
// covered box keeps >= R cells from its faces)
void launch_hoz_fas(const double* u, double* f, const int* n, int periodic, const int* lo, const int* cn, double h,
                    int order, hipStream_t st);
void launch_hoz_prolong(double* u, const HozPatch& P, const double* pu, const double* uold, hipStream_t st);
void launch_hoz_restrict(const double* v, const HozPatch& P, double* pv, hipStream_t st);
// partial sums over the cells outside the box lo + [0, cn) (cn = 0: every cell) into
// part[0 .. kHozParts): MODE 0 v^2; MODE 1 r^2 of a patch (g its ghosts); MODE 2 r^2 of the base
constexpr int kHozParts = 2048;
void launch_hoz_psum(int mode, const double* v, const double* f, const double* g, const int* n, const int* lo,
                     const int* cn, double h, int order, double* part, hipStream_t st);

}  // namespace mgic
