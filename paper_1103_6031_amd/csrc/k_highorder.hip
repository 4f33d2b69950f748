// Periodic FAS multigrid with the fourth- and sixth-order Laplacians of Table 1 (Section 3.2).
//
// The 1-D stencil of order 2R (R = 1, 2, 3) is summed over the three axes: 7, 13 or 19 points.
// Every level of the V-cycle uses the same operator.  The grid is n^3 with n a power of two, in
// natural [x][y][z] order, z contiguous; offsets wrap by masking with n - 1.
//
// Red-black with a radius-R stencil: cells two apart along an axis share a colour and couple, so
// a half-sweep updates every cell of its colour from the values before the half-sweep (Jacobi
// within the colour, Gauss-Seidel between colours).  That makes the half-sweep out of place: it
// reads `in` and writes every cell of `out` (its colour updated, the other copied), so two
// half-sweeps return the iterate to the buffer it started in.  The update solves the cell's own
// equation for its centre value: u <- (h^2 f - sum_s w_s sum_axes (u[i-s] + u[i+s])) / (3 w_0).
//
// FP64 throughout; the arithmetic is the oracle's up to summation order.

#include "mg_internal.h"

namespace mgic {

namespace {

template <int R> struct HoW;
template <> struct HoW<1> { static constexpr double w0 = -2.0, w1 = 1.0, w2 = 0.0, w3 = 0.0; };
template <> struct HoW<2> {
    static constexpr double w0 = -30.0 / 12, w1 = 16.0 / 12, w2 = -1.0 / 12, w3 = 0.0;
};
template <> struct HoW<3> {
    static constexpr double w0 = -490.0 / 180, w1 = 270.0 / 180, w2 = -27.0 / 180, w3 = 2.0 / 180;
};

template <int R>
__device__ __forceinline__ double ho_w(int s) {
    return s == 1 ? HoW<R>::w1 : (s == 2 ? HoW<R>::w2 : HoW<R>::w3);
}

__device__ __forceinline__ unsigned ho_idx(unsigned x, unsigned y, unsigned z, int lg) {
    return (x << (2 * lg)) | (y << lg) | z;
}

// sum_{s=1..R} w_s (((x-s) + (x+s)) + ((y-s) + (y+s))) + ((z-s) + (z+s))), periodic
template <int R>
__device__ __forceinline__ double ho_off(const double* __restrict__ u, unsigned x, unsigned y, unsigned z, int lg,
                                         unsigned m) {
    double acc = 0.0;
#pragma unroll
    for (int s = 1; s <= R; ++s) {
        const double px = u[ho_idx((x - s) & m, y, z, lg)] + u[ho_idx((x + s) & m, y, z, lg)];
        const double py = u[ho_idx(x, (y - s) & m, z, lg)] + u[ho_idx(x, (y + s) & m, z, lg)];
        const double pz = u[ho_idx(x, y, (z - s) & m, lg)] + u[ho_idx(x, y, (z + s) & m, lg)];
        acc += ho_w<R>(s) * ((px + py) + pz);
    }
    return acc;
}

// Block order: consecutive blocks go to the 8 XCDs in turn.  Blocks that hold x-neighbouring
// planes are a multiple of 8 apart and already share an XCD's L2; the y-neighbour rows of a
// block's edge rows belong to the next blocks.  Within groups of 8k blocks, k consecutive ones
// go to one XCD (k = 8 from 128 blocks per plane, 4 from 32; the order is unchanged below).
__device__ __forceinline__ unsigned ho_xcd_group(unsigned b, int lgbpp) {
    if (lgbpp < 5) return b;
    const int lk = lgbpp >= 7 ? 3 : 2;
    const unsigned G = 8u << lk;
    return (b & ~(G - 1)) | ((b & 7u) << lk) | ((b >> 3) & ((1u << lk) - 1));
}

// one thread per pair of z-neighbours (2p, 2p + 1): exactly one of them has the colour, so every
// lane computes one update; the pair is read and written as one 16-byte access
template <int R>
__global__ __launch_bounds__(kBlock) void k_ho_half(const double* __restrict__ in, double* __restrict__ out,
                                                    const double* __restrict__ f, int lg, double h2, int colour) {
    const unsigned p = ho_xcd_group(blockIdx.x, 2 * lg - 9) * blockDim.x + threadIdx.x;
    if (p >= (1u << (3 * lg - 1))) return;
    const unsigned t0 = 2 * p, m = (1u << lg) - 1, z0 = t0 & m, y = (t0 >> lg) & m, x = t0 >> (2 * lg);
    const unsigned q = (x + y + (unsigned)colour) & 1u;   // (x + y + z0 + q) & 1 == colour
    const double2 cur = *(const double2*)(in + t0);
    const double v = (h2 * f[t0 + q] - ho_off<R>(in, x, y, z0 + q, lg, m)) / (3.0 * HoW<R>::w0);
    *(double2*)(out + t0) = q ? make_double2(cur.x, v) : make_double2(v, cur.y);
}

// r = f - L u for the two cells (x, y, z0) and (x, y, z0 + 1), z0 even, from 16-byte loads: the
// pairs of the x- and y-neighbour rows hold both cells' neighbours, and one run of pairs from
// z0 - 2J to z0 + 2J + 1 (J = ceil(R / 2)) holds their z-neighbours.  Same arithmetic as ho_off.
template <int R>
__device__ __forceinline__ double2 ho_pair_resid(const double* __restrict__ u, const double* __restrict__ f,
                                                 unsigned x, unsigned y, unsigned z0, int lg, unsigned m,
                                                 double h2, double2* own) {
    constexpr int J = (R + 1) / 2;
    double zr[4 * J + 2];
#pragma unroll
    for (int j = -J; j <= J; ++j) {
        const double2 v = *(const double2*)(u + ho_idx(x, y, (z0 + 2 * j) & m, lg));
        zr[2 * (j + J)] = v.x;
        zr[2 * (j + J) + 1] = v.y;
    }
    double acc[2] = {0.0, 0.0};
#pragma unroll
    for (int s = 1; s <= R; ++s) {
        const double2 xm = *(const double2*)(u + ho_idx((x - s) & m, y, z0, lg));
        const double2 xp = *(const double2*)(u + ho_idx((x + s) & m, y, z0, lg));
        const double2 ym = *(const double2*)(u + ho_idx(x, (y - s) & m, z0, lg));
        const double2 yp = *(const double2*)(u + ho_idx(x, (y + s) & m, z0, lg));
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const double px = (c ? xm.y : xm.x) + (c ? xp.y : xp.x);
            const double py = (c ? ym.y : ym.x) + (c ? yp.y : yp.x);
            const double pz = zr[2 * J + c - s] + zr[2 * J + c + s];
            acc[c] += ho_w<R>(s) * ((px + py) + pz);
        }
    }
    const double2 fv = *(const double2*)(f + ho_idx(x, y, z0, lg));
    const double u0 = zr[2 * J], u1 = zr[2 * J + 1];
    *own = make_double2(u0, u1);
    return make_double2(fv.x - (acc[0] + 3.0 * HoW<R>::w0 * u0) / h2, fv.y - (acc[1] + 3.0 * HoW<R>::w0 * u1) / h2);
}

// steps 3-5 for one coarse cell: the mean of the 8 children's residuals and of their values
template <int R>
__global__ __launch_bounds__(kBlock) void k_ho_resid_restrict(const double* __restrict__ u, const double* __restrict__ f,
                                                              double* __restrict__ uc, double* __restrict__ uold,
                                                              double* __restrict__ rc, int lgc, double h2) {
    const unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (1u << (3 * lgc))) return;
    const int lg = lgc + 1;
    const unsigned mc = (1u << lgc) - 1, m = (1u << lg) - 1;
    const unsigned Z = t & mc, Y = (t >> lgc) & mc, X = t >> (2 * lgc);
    double rs = 0.0, us = 0.0;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {   // children (2X + a, 2Y + b, 2Z + c), c = 0, 1
            double2 uv;
            const double2 r = ho_pair_resid<R>(u, f, 2 * X + a, 2 * Y + b, 2 * Z, lg, m, h2, &uv);
            rs += r.x;
            us += uv.x;
            rs += r.y;
            us += uv.y;
        }
    const double um = us * 0.125;
    uc[t] = um;
    uold[t] = um;
    rc[t] = rs * 0.125;
}

// step 6: fc = rc + L uc, in place over rc
template <int R>
__global__ __launch_bounds__(kBlock) void k_ho_fas(const double* __restrict__ uc, double* __restrict__ fc, int lgc,
                                                   double h2) {
    const unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (1u << (3 * lgc))) return;
    const unsigned m = (1u << lgc) - 1, z = t & m, y = (t >> lgc) & m, x = t >> (2 * lgc);
    fc[t] = fc[t] + (ho_off<R>(uc, x, y, z, lgc, m) + 3.0 * HoW<R>::w0 * uc[t]) / h2;
}

// step 8: u += inject(uc - uold)
__global__ __launch_bounds__(kBlock) void k_ho_prolong(double* __restrict__ u, const double* __restrict__ uc,
                                                       const double* __restrict__ uold, int lg) {
    const unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (1u << (3 * lg))) return;
    const int lgc = lg - 1;
    const unsigned m = (1u << lg) - 1, z = t & m, y = (t >> lg) & m, x = t >> (2 * lg);
    const unsigned p = ho_idx(x >> 1, y >> 1, z >> 1, lgc);
    u[t] = u[t] + (uc[p] - uold[p]);
}

__global__ __launch_bounds__(kBlock) void k_ho_fill(double* __restrict__ a, unsigned n, double v) {
    const unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) a[t] = v;
}

// deterministic block sum (wave64 shuffle, then the waves in order); valid on thread 0
__device__ double ho_block_sum(double v) {
    __shared__ double s_w[kBlock / 64];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) s_w[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) r += s_w[k];
    return r;
}

// partial sums over a fixed grid: MODE 0 sum of a; MODE 1 sum of squares of r = f - L u
template <int R, int MODE>
__global__ __launch_bounds__(kBlock) void k_ho_psum(const double* __restrict__ a, const double* __restrict__ f,
                                                    int lg, double h2, double* __restrict__ part) {
    const unsigned n = 1u << (3 * lg), m = (1u << lg) - 1;
    double acc = 0.0;
    if (MODE == 0) {
        for (unsigned t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) acc += a[t];
    } else {   // pairs of z-neighbours (n is even)
        for (unsigned p = blockIdx.x * blockDim.x + threadIdx.x; p < n / 2; p += gridDim.x * blockDim.x) {
            const unsigned t = 2 * p, z = t & m, y = (t >> lg) & m, x = t >> (2 * lg);
            double2 uv;
            const double2 r = ho_pair_resid<R>(a, f, x, y, z, lg, m, h2, &uv);
            acc += r.x * r.x;
            acc += r.y * r.y;
        }
    }
    const double s = ho_block_sum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// out = a - (*sum) / n, with the partial sums of out^2
__global__ __launch_bounds__(kBlock) void k_ho_sub(const double* a, const double* __restrict__ sum,
                                                   double* out, int lg, double* __restrict__ part) {
    const unsigned n = 1u << (3 * lg);
    const double mean = *sum / (double)n;
    double acc = 0.0;
    for (unsigned t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
        const double v = a[t] - mean;
        out[t] = v;
        acc += v * v;
    }
    const double s = ho_block_sum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// out[0] = sum of part[0..cnt) in a fixed order (one block)
__global__ __launch_bounds__(kBlock) void k_ho_reduce(const double* __restrict__ part, int cnt,
                                                      double* __restrict__ out) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < cnt; i += blockDim.x) acc += part[i];
    const double s = ho_block_sum(acc);
    if (threadIdx.x == 0) out[0] = s;
}

int ho_parts(int lg) {   // blocks of the reductions: fixed by the size, at most kHoParts
    const size_t n = (size_t)1 << (3 * lg);
    return grid_for(n, kBlock * 8, kHoParts);
}

}  // namespace

#define HO_DISPATCH(order, KERNEL, GRID, ...)                                                  \
    do {                                                                                       \
        if ((order) == 2) KERNEL<1><<<(GRID), kBlock, 0, st>>>(__VA_ARGS__);                   \
        else if ((order) == 4) KERNEL<2><<<(GRID), kBlock, 0, st>>>(__VA_ARGS__);              \
        else KERNEL<3><<<(GRID), kBlock, 0, st>>>(__VA_ARGS__);                                \
    } while (0)

void launch_ho_half(const double* in, double* out, const double* f, int lg, double h, int order, int colour,
                    hipStream_t st, hipEvent_t ea, hipEvent_t eb) {
    const int g = grid_for((size_t)1 << (3 * lg - 1));   // pairs of cells (lg >= 1)
    if (ea) (void)hipEventRecord(ea, st);
    HO_DISPATCH(order, k_ho_half, g, in, out, f, lg, h * h, colour);
    if (eb) (void)hipEventRecord(eb, st);
}

void launch_ho_resid_restrict(const double* u, const double* f, double* uc, double* uold, double* rc, int lgc,
                              double h, int order, hipStream_t st) {
    HO_DISPATCH(order, k_ho_resid_restrict, grid_for((size_t)1 << (3 * lgc)), u, f, uc, uold, rc, lgc, h * h);
}

void launch_ho_fas(const double* uc, double* fc, int lgc, double hc, int order, hipStream_t st) {
    HO_DISPATCH(order, k_ho_fas, grid_for((size_t)1 << (3 * lgc)), uc, fc, lgc, hc * hc);
}

void launch_ho_prolong(double* u, const double* uc, const double* uold, int lg, hipStream_t st) {
    k_ho_prolong<<<grid_for((size_t)1 << (3 * lg)), kBlock, 0, st>>>(u, uc, uold, lg);
}

void launch_ho_fill(double* a, int lg, double v, hipStream_t st) {
    const unsigned n = 1u << (3 * lg);
    k_ho_fill<<<grid_for(n), kBlock, 0, st>>>(a, n, v);
}

void launch_ho_sum(const double* a, int lg, double* part, double* out, hipStream_t st) {
    const int nb = ho_parts(lg);
    k_ho_psum<1, 0><<<nb, kBlock, 0, st>>>(a, nullptr, lg, 1.0, part);
    k_ho_reduce<<<1, kBlock, 0, st>>>(part, nb, out);
}

void launch_ho_sub(const double* a, const double* sum, double* out, int lg, double* part, double* sumsq,
                   hipStream_t st) {
    const int nb = ho_parts(lg);
    k_ho_sub<<<nb, kBlock, 0, st>>>(a, sum, out, lg, part);
    k_ho_reduce<<<1, kBlock, 0, st>>>(part, nb, sumsq);
}

void launch_ho_rnorm(const double* u, const double* f, int lg, double h, int order, double* part, double* out,
                     hipStream_t st) {
    const int nb = ho_parts(lg);
    const double h2 = h * h;
    if (order == 2) k_ho_psum<1, 1><<<nb, kBlock, 0, st>>>(u, f, lg, h2, part);
    else if (order == 4) k_ho_psum<2, 1><<<nb, kBlock, 0, st>>>(u, f, lg, h2, part);
    else k_ho_psum<3, 1><<<nb, kBlock, 0, st>>>(u, f, lg, h2, part);
    k_ho_reduce<<<1, kBlock, 0, st>>>(part, nb, out);
}

}  // namespace mgic
