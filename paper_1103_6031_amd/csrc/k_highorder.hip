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
// The V-cycle kernels take the element type T: FP64, or FP32 for the inner cycles of the
// mixed-precision solve, whose FP64 residual (k_ho_resid32) and correction (k_ho_add32) are
// separate kernels.  The FP64 arithmetic is the oracle's up to summation order.

#include <algorithm>

#include "mg_internal.h"

namespace mgic {

namespace {

template <class T> struct HoV2;
template <> struct HoV2<double> { using type = double2; };
template <> struct HoV2<float> { using type = float2; };
template <class T> using v2_t = typename HoV2<T>::type;
template <class T>
__device__ __forceinline__ v2_t<T> mk2(T a, T b) {
    v2_t<T> r;
    r.x = a;
    r.y = b;
    return r;
}

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
template <int R, class T>
__device__ __forceinline__ T ho_off(const T* __restrict__ u, unsigned x, unsigned y, unsigned z, int lg,
                                    unsigned m) {
    T acc = 0;
#pragma unroll
    for (int s = 1; s <= R; ++s) {
        const T px = u[ho_idx((x - s) & m, y, z, lg)] + u[ho_idx((x + s) & m, y, z, lg)];
        const T py = u[ho_idx(x, (y - s) & m, z, lg)] + u[ho_idx(x, (y + s) & m, z, lg)];
        const T pz = u[ho_idx(x, y, (z - s) & m, lg)] + u[ho_idx(x, y, (z + s) & m, lg)];
        acc += (T)ho_w<R>(s) * ((px + py) + pz);
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
    if (gridDim.x & (G - 1)) return b;   // the permutation needs whole groups
    return (b & ~(G - 1)) | ((b & 7u) << lk) | ((b >> 3) & ((1u << lk) - 1));
}

// one thread per pair of z-neighbours (2p, 2p + 1): exactly one of them has the colour, so every
// lane computes one update; the pair is read and written as one 16-byte access
template <int R, class T>
__global__ __launch_bounds__(kBlock) void k_ho_half(const T* __restrict__ in, T* __restrict__ out,
                                                    const T* __restrict__ f, int lg, T h2, int colour) {
    const unsigned p = ho_xcd_group(blockIdx.x, 2 * lg - 9) * blockDim.x + threadIdx.x;
    if (p >= (1u << (3 * lg - 1))) return;
    const unsigned t0 = 2 * p, m = (1u << lg) - 1, z0 = t0 & m, y = (t0 >> lg) & m, x = t0 >> (2 * lg);
    const unsigned q = (x + y + (unsigned)colour) & 1u;   // (x + y + z0 + q) & 1 == colour
    const v2_t<T> cur = *(const v2_t<T>*)(in + t0);
    const T v = (h2 * f[t0 + q] - ho_off<R>(in, x, y, z0 + q, lg, m)) / ((T)3 * (T)HoW<R>::w0);
    *(v2_t<T>*)(out + t0) = q ? mk2<T>(cur.x, v) : mk2<T>(v, cur.y);
}

// The same half-sweep with the y and z neighbours from LDS: a block owns rows y0 .. y0 + kHoTy - 1
// of one x plane and stages them with R halo rows on each side (all z, wrapped in y) in LDS; the
// 2R x-neighbours and f come from memory.  About 2R + 3 global loads per update instead of
// 6R + 2; the sums are formed in the order of ho_off, so the bits are the same.  Blocks of one
// plane are consecutive; the blocks of x-neighbouring planes are n / kHoTy apart, a multiple of 8
// from n = 64 on, so they share an XCD (and its L2).  For 16 <= n <= 256.  Eight rows per block
// (29 KB of LDS at 256^3 FP64, order 6) measured best: 16 rows 116 us, 8 rows 109 us, 4 rows
// 111 us at 256^3 (order 6, FP64): the halo rows cost less than the blocks per CU gained.
constexpr int kHoTy = 8;

// Rows y0 - R .. y0 + kHoTy + R - 1 of plane x (all z, wrapped in y) into rows[kHoTy + 2R][n], as
// 16-byte pairs; each thread's loads go in batches of 8 before their LDS writes (so that they
// are in flight together).  The caller synchronises the block afterwards.
template <int R, class T>
__device__ __forceinline__ void ho_stage_rows(T* __restrict__ rows, const T* __restrict__ in, unsigned x,
                                              unsigned y0, int lg) {
    const unsigned n = 1u << lg, m = n - 1, nh = n >> 1;
    constexpr int kBatch = 8;
    const unsigned npairs = (unsigned)(kHoTy + 2 * R) * nh;
    for (unsigned t0 = threadIdx.x; t0 < npairs; t0 += kBatch * blockDim.x) {
        v2_t<T> v[kBatch];
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
            const unsigned t = t0 + k * blockDim.x;
            v[k] = mk2<T>((T)0, (T)0);
            if (t < npairs) {
                const unsigned r = t / nh, pz = t - r * nh;
                const unsigned y = (y0 + r - R) & m;
                v[k] = *(const v2_t<T>*)(in + ho_idx(x, y, 2 * pz, lg));
            }
        }
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
            const unsigned t = t0 + k * blockDim.x;
            if (t < npairs) {
                const unsigned r = t / nh, pz = t - r * nh;
                *(v2_t<T>*)(rows + r * n + 2 * pz) = v[k];
            }
        }
    }
}

template <int R, class T>
__global__ __launch_bounds__(kBlock) void k_ho_half_lds(const T* __restrict__ in, T* __restrict__ out,
                                                        const T* __restrict__ f, int lg, T h2, int colour) {
    extern __shared__ __align__(16) unsigned char ho_smem[];
    T* rows = (T*)ho_smem;                          // [kHoTy + 2R][n]
    const unsigned n = 1u << lg, m = n - 1, nh = n >> 1;
    const unsigned tiles = n / kHoTy;
    const unsigned bl = ho_xcd_group(blockIdx.x, lg - 3);   // consecutive tiles of a plane on one XCD
    const unsigned x = bl / tiles, y0 = (bl - x * tiles) * kHoTy;
    ho_stage_rows<R, T>(rows, in, x, y0, lg);
    __syncthreads();
    const unsigned pairs = (unsigned)kHoTy * nh;
    for (unsigned t = threadIdx.x; t < pairs; t += blockDim.x) {
        const unsigned ry = t / nh, pz = t - ry * nh;
        const unsigned y = y0 + ry, z0 = 2 * pz;
        const unsigned q = (x + y + (unsigned)colour) & 1u;
        const unsigned z = z0 + q;
        const T* row = rows + (ry + R) * n;
        T acc = 0;
#pragma unroll
        for (int s = 1; s <= R; ++s) {
            const T px = in[ho_idx((x - s) & m, y, z, lg)] + in[ho_idx((x + s) & m, y, z, lg)];
            const T py = row[(int)z - s * (int)n] + row[(int)z + s * (int)n];   // rows y - s, y + s
            const T pz_ = row[(z - s) & m] + row[(z + s) & m];
            acc += (T)ho_w<R>(s) * ((px + py) + pz_);
        }
        const v2_t<T> cur = *(const v2_t<T>*)(row + z0);
        const T v = (h2 * f[ho_idx(x, y, z, lg)] - acc) / ((T)3 * (T)HoW<R>::w0);
        *(v2_t<T>*)(out + ho_idx(x, y, z0, lg)) = q ? mk2<T>(cur.x, v) : mk2<T>(v, cur.y);
    }
}

// r = f - L u for the two cells (x, y, z0) and (x, y, z0 + 1), z0 even, from 16-byte loads: the
// pairs of the x- and y-neighbour rows hold both cells' neighbours, and one run of pairs from
// z0 - 2J to z0 + 2J + 1 (J = ceil(R / 2)) holds their z-neighbours.  Same arithmetic as ho_off.
template <int R, class T>
__device__ __forceinline__ v2_t<T> ho_pair_resid(const T* __restrict__ u, const T* __restrict__ f,
                                                 unsigned x, unsigned y, unsigned z0, int lg, unsigned m,
                                                 T h2, v2_t<T>* own) {
    constexpr int J = (R + 1) / 2;
    T zr[4 * J + 2];
#pragma unroll
    for (int j = -J; j <= J; ++j) {
        const v2_t<T> v = *(const v2_t<T>*)(u + ho_idx(x, y, (z0 + 2 * j) & m, lg));
        zr[2 * (j + J)] = v.x;
        zr[2 * (j + J) + 1] = v.y;
    }
    T acc[2] = {0, 0};
#pragma unroll
    for (int s = 1; s <= R; ++s) {
        const v2_t<T> xm = *(const v2_t<T>*)(u + ho_idx((x - s) & m, y, z0, lg));
        const v2_t<T> xp = *(const v2_t<T>*)(u + ho_idx((x + s) & m, y, z0, lg));
        const v2_t<T> ym = *(const v2_t<T>*)(u + ho_idx(x, (y - s) & m, z0, lg));
        const v2_t<T> yp = *(const v2_t<T>*)(u + ho_idx(x, (y + s) & m, z0, lg));
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const T px = (c ? xm.y : xm.x) + (c ? xp.y : xp.x);
            const T py = (c ? ym.y : ym.x) + (c ? yp.y : yp.x);
            const T pz = zr[2 * J + c - s] + zr[2 * J + c + s];
            acc[c] += (T)ho_w<R>(s) * ((px + py) + pz);
        }
    }
    const v2_t<T> fv = *(const v2_t<T>*)(f + ho_idx(x, y, z0, lg));
    const T u0 = zr[2 * J], u1 = zr[2 * J + 1];
    const T w0x3 = (T)3 * (T)HoW<R>::w0;
    *own = mk2<T>(u0, u1);
    return mk2<T>(fv.x - (acc[0] + w0x3 * u0) / h2, fv.y - (acc[1] + w0x3 * u1) / h2);
}

// ho_pair_resid with the y and z neighbours from rows staged by ho_stage_rows: `row` is the
// staged row of y (R rows after the first staged one); the 2R x-neighbour pairs and f come from
// memory.  The same arithmetic in the same order, so the same bits.
template <int R, class T>
__device__ __forceinline__ v2_t<T> ho_pair_resid_lds(const T* __restrict__ row, const T* __restrict__ u,
                                                     const T* __restrict__ f, unsigned x, unsigned y,
                                                     unsigned z0, int lg, T h2, v2_t<T>* own) {
    constexpr int J = (R + 1) / 2;
    const unsigned n = 1u << lg, m = n - 1;
    T zr[4 * J + 2];
#pragma unroll
    for (int j = -J; j <= J; ++j) {
        const v2_t<T> v = *(const v2_t<T>*)(row + ((z0 + 2 * j) & m));
        zr[2 * (j + J)] = v.x;
        zr[2 * (j + J) + 1] = v.y;
    }
    T acc[2] = {0, 0};
#pragma unroll
    for (int s = 1; s <= R; ++s) {
        const v2_t<T> xm = *(const v2_t<T>*)(u + ho_idx((x - s) & m, y, z0, lg));
        const v2_t<T> xp = *(const v2_t<T>*)(u + ho_idx((x + s) & m, y, z0, lg));
        const v2_t<T> ym = *(const v2_t<T>*)(row - s * (int)n + z0);   // rows y - s, y + s
        const v2_t<T> yp = *(const v2_t<T>*)(row + s * (int)n + z0);
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const T px = (c ? xm.y : xm.x) + (c ? xp.y : xp.x);
            const T py = (c ? ym.y : ym.x) + (c ? yp.y : yp.x);
            const T pz = zr[2 * J + c - s] + zr[2 * J + c + s];
            acc[c] += (T)ho_w<R>(s) * ((px + py) + pz);
        }
    }
    const v2_t<T> fv = *(const v2_t<T>*)(f + ho_idx(x, y, z0, lg));
    const T u0 = zr[2 * J], u1 = zr[2 * J + 1];
    const T w0x3 = (T)3 * (T)HoW<R>::w0;
    *own = mk2<T>(u0, u1);
    return mk2<T>(fv.x - (acc[0] + w0x3 * u0) / h2, fv.y - (acc[1] + w0x3 * u1) / h2);
}

// steps 3-5 for one coarse cell: the mean of the 8 children's residuals and of their values
template <int R, class T>
__global__ __launch_bounds__(kBlock) void k_ho_resid_restrict(const T* __restrict__ u, const T* __restrict__ f,
                                                              T* __restrict__ uc, T* __restrict__ uold,
                                                              T* __restrict__ rc, int lgc, T h2) {
    const unsigned t = ho_xcd_group(blockIdx.x, 2 * lgc - 8) * blockDim.x + threadIdx.x;
    if (t >= (1u << (3 * lgc))) return;
    const int lg = lgc + 1;
    const unsigned mc = (1u << lgc) - 1, m = (1u << lg) - 1;
    const unsigned Z = t & mc, Y = (t >> lgc) & mc, X = t >> (2 * lgc);
    T rs = 0, us = 0;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {   // children (2X + a, 2Y + b, 2Z + c), c = 0, 1
            v2_t<T> uv;
            const v2_t<T> r = ho_pair_resid<R, T>(u, f, 2 * X + a, 2 * Y + b, 2 * Z, lg, m, h2, &uv);
            rs += r.x;
            us += uv.x;
            rs += r.y;
            us += uv.y;
        }
    const T um = us * (T)0.125;
    uc[t] = um;
    uold[t] = um;
    rc[t] = rs * (T)0.125;
}

// k_ho_resid_restrict with the fine rows staged in LDS: a block owns coarse plane X and coarse
// rows Y0 .. Y0 + kHoTy / 2 - 1 (fine rows y0 = 2 Y0 .. y0 + kHoTy - 1), stages fine plane 2X, then
// 2X + 1, into the same rows (ho_stage_rows), and each thread keeps the sums of its coarse cells
// over both planes: children in the order of k_ho_resid_restrict, so the same bits.  For fine
// sizes 16 <= n <= 256 (at most 2 coarse cells per thread).
template <int R, class T>
__global__ __launch_bounds__(kBlock) void k_ho_resid_restrict_lds(const T* __restrict__ u, const T* __restrict__ f,
                                                                  T* __restrict__ uc, T* __restrict__ uold,
                                                                  T* __restrict__ rc, int lgc, T h2) {
    extern __shared__ __align__(16) unsigned char ho_smem[];
    T* rows = (T*)ho_smem;                           // [kHoTy + 2R][n]
    constexpr int kC = 2;
    const int lg = lgc + 1;
    const unsigned n = 1u << lg, nc = n >> 1;
    const unsigned tiles = n / kHoTy;
    const unsigned bl = ho_xcd_group(blockIdx.x, lg - 3);
    const unsigned X = bl / tiles, y0 = (bl - X * tiles) * kHoTy;
    const unsigned cells = (unsigned)(kHoTy / 2) * nc;
    T rs[kC], us[kC];
#pragma unroll
    for (int k = 0; k < kC; ++k) rs[k] = us[k] = (T)0;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        if (a) __syncthreads();                      // every read of plane 2X done
        ho_stage_rows<R, T>(rows, u, 2 * X + a, y0, lg);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kC; ++k) {
            const unsigned c = threadIdx.x + k * blockDim.x;
            if (c < cells) {
                const unsigned yl = c / nc, Z = c - yl * nc;
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    const unsigned ry = 2 * yl + b;
                    v2_t<T> uv;
                    const v2_t<T> r = ho_pair_resid_lds<R, T>(rows + (ry + R) * n, u, f, 2 * X + a, y0 + ry,
                                                              2 * Z, lg, h2, &uv);
                    rs[k] += r.x;
                    us[k] += uv.x;
                    rs[k] += r.y;
                    us[k] += uv.y;
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < kC; ++k) {
        const unsigned c = threadIdx.x + k * blockDim.x;
        if (c < cells) {
            const unsigned yl = c / nc, Z = c - yl * nc;
            const unsigned t = ho_idx(X, y0 / 2 + yl, Z, lgc);
            const T um = us[k] * (T)0.125;
            uc[t] = um;
            uold[t] = um;
            rc[t] = rs[k] * (T)0.125;
        }
    }
}

// step 6: fc = rc + L uc, in place over rc
template <int R, class T>
__global__ __launch_bounds__(kBlock) void k_ho_fas(const T* __restrict__ uc, T* __restrict__ fc, int lgc, T h2) {
    const unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (1u << (3 * lgc))) return;
    const unsigned m = (1u << lgc) - 1, z = t & m, y = (t >> lgc) & m, x = t >> (2 * lgc);
    fc[t] = fc[t] + (ho_off<R>(uc, x, y, z, lgc, m) + (T)3 * (T)HoW<R>::w0 * uc[t]) / h2;
}

// step 8: u += inject(uc - uold)
template <class T>
__global__ __launch_bounds__(kBlock) void k_ho_prolong(T* __restrict__ u, const T* __restrict__ uc,
                                                       const T* __restrict__ uold, int lg) {
    const unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (1u << (3 * lg))) return;
    const int lgc = lg - 1;
    const unsigned m = (1u << lg) - 1, z = t & m, y = (t >> lg) & m, x = t >> (2 * lg);
    const unsigned p = ho_idx(x >> 1, y >> 1, z >> 1, lgc);
    u[t] = u[t] + (uc[p] - uold[p]);
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_ho_fill(T* __restrict__ a, unsigned n, T v) {
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
    // block bl takes the pairs (and stores the partial) of block bl in dispatch order, so the
    // partial sums are the same; bl groups consecutive rows of a plane on one XCD
    const unsigned bl = MODE == 0 ? blockIdx.x : ho_xcd_group(blockIdx.x, 2 * lg - 9);
    if (MODE == 0) {
        for (unsigned t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) acc += a[t];
    } else {   // pairs of z-neighbours (n is even)
        for (unsigned p = bl * blockDim.x + threadIdx.x; p < n / 2; p += gridDim.x * blockDim.x) {
            const unsigned t = 2 * p, z = t & m, y = (t >> lg) & m, x = t >> (2 * lg);
            double2 uv;
            const double2 r = ho_pair_resid<R, double>(a, f, x, y, z, lg, m, h2, &uv);
            acc += r.x * r.x;
            acc += r.y * r.y;
        }
    }
    const double s = ho_block_sum(acc);
    if (threadIdx.x == 0) part[bl] = s;
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

// mixed precision: r32 = (float)(f - L u) in FP64, with the partial sums of r^2 (pairs of cells)
template <int R>
__global__ __launch_bounds__(kBlock) void k_ho_resid32(const double* __restrict__ u, const double* __restrict__ f,
                                                       float* __restrict__ r32, int lg, double h2,
                                                       double* __restrict__ part) {
    const unsigned n = 1u << (3 * lg), m = (1u << lg) - 1;
    double acc = 0.0;
    const unsigned bl = ho_xcd_group(blockIdx.x, 2 * lg - 9);   // as in k_ho_psum
    for (unsigned p = bl * blockDim.x + threadIdx.x; p < n / 2; p += gridDim.x * blockDim.x) {
        const unsigned t = 2 * p, z = t & m, y = (t >> lg) & m, x = t >> (2 * lg);
        double2 uv;
        const double2 r = ho_pair_resid<R, double>(u, f, x, y, z, lg, m, h2, &uv);
        *(float2*)(r32 + t) = make_float2((float)r.x, (float)r.y);
        acc += r.x * r.x;
        acc += r.y * r.y;
    }
    const double s = ho_block_sum(acc);
    if (threadIdx.x == 0) part[bl] = s;
}

// r = f - L u over a block's rows, staged as in k_ho_half_lds (rows y0 - R .. y0 + kHoTy + R - 1 of
// plane x in LDS; the 2R x-neighbour pairs and f from memory), with the arithmetic of
// ho_pair_resid, so every r has the same bits.  The block's sum of r^2 goes to part at its tile
// index (kHoTy rows of a plane, n^2 / kHoTy tiles in all); kR32 also writes r as FP32 (the
// right-hand side of the mixed-precision inner cycles).  For 16 <= n <= 256, like the half-sweep.
template <int R, bool kR32>
__global__ __launch_bounds__(kBlock) void k_ho_resid_lds(const double* __restrict__ u, const double* __restrict__ f,
                                                         float* __restrict__ r32, int lg, double h2,
                                                         double* __restrict__ part) {
    extern __shared__ __align__(16) unsigned char ho_smem[];
    double* rows = (double*)ho_smem;                 // [kHoTy + 2R][n]
    const unsigned n = 1u << lg, nh = n >> 1;
    const unsigned tiles = n / kHoTy;
    const unsigned bl = ho_xcd_group(blockIdx.x, lg - 3);
    const unsigned x = bl / tiles, y0 = (bl - x * tiles) * kHoTy;
    ho_stage_rows<R, double>(rows, u, x, y0, lg);
    __syncthreads();
    double acc2 = 0.0;
    const unsigned pairs = (unsigned)kHoTy * nh;
    for (unsigned t = threadIdx.x; t < pairs; t += blockDim.x) {
        const unsigned ry = t / nh, pz = t - ry * nh;
        const unsigned y = y0 + ry, z0 = 2 * pz;
        double2 uv;
        const double2 r = ho_pair_resid_lds<R, double>(rows + (ry + R) * n, u, f, x, y, z0, lg, h2, &uv);
        const double r0 = r.x, r1 = r.y;
        if constexpr (kR32) *(float2*)(r32 + ho_idx(x, y, z0, lg)) = make_float2((float)r0, (float)r1);
        acc2 += r0 * r0;
        acc2 += r1 * r1;
    }
    const double s = ho_block_sum(acc2);
    if (threadIdx.x == 0) part[bl] = s;
}

// mixed precision: u += e (the FP32 correction)
__global__ __launch_bounds__(kBlock) void k_ho_add32(double* __restrict__ u, const float* __restrict__ e, int lg) {
    const unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < (1u << (3 * lg))) u[t] = u[t] + (double)e[t];
}

int ho_parts(int lg) {   // blocks of the reductions: fixed by the size, at most kHoParts
    const size_t n = (size_t)1 << (3 * lg);
    return grid_for(n, kBlock * 8, kHoParts);
}

}  // namespace

#define HO_DISPATCH(order, KERNEL, T, GRID, ...)                                               \
    do {                                                                                       \
        if ((order) == 2) KERNEL<1, T><<<(GRID), kBlock, 0, st>>>(__VA_ARGS__);                \
        else if ((order) == 4) KERNEL<2, T><<<(GRID), kBlock, 0, st>>>(__VA_ARGS__);           \
        else KERNEL<3, T><<<(GRID), kBlock, 0, st>>>(__VA_ARGS__);                             \
    } while (0)

template <class T>
void launch_ho_half(const T* in, T* out, const T* f, int lg, double h, int order, int colour, hipStream_t st,
                    hipEvent_t ea, hipEvent_t eb) {
    if (ea) (void)hipEventRecord(ea, st);
    if (lg >= 4 && lg <= 8) {   // 16^3 .. 256^3: y and z neighbours from LDS
        const unsigned n = 1u << lg;
        const unsigned blocks = n * (n / kHoTy);
        const T h2 = (T)(h * h);
        const int R = order / 2;
        const size_t lds = (size_t)(kHoTy + 2 * R) * n * sizeof(T);
        if (order == 2) k_ho_half_lds<1, T><<<blocks, kBlock, lds, st>>>(in, out, f, lg, h2, colour);
        else if (order == 4) k_ho_half_lds<2, T><<<blocks, kBlock, lds, st>>>(in, out, f, lg, h2, colour);
        else k_ho_half_lds<3, T><<<blocks, kBlock, lds, st>>>(in, out, f, lg, h2, colour);
    } else {
        const int g = grid_for((size_t)1 << (3 * lg - 1));   // pairs of cells (lg >= 1)
        HO_DISPATCH(order, k_ho_half, T, g, in, out, f, lg, (T)(h * h), colour);
    }
    if (eb) (void)hipEventRecord(eb, st);
}

template <class T>
void launch_ho_resid_restrict(const T* u, const T* f, T* uc, T* uold, T* rc, int lgc, double h, int order,
                              hipStream_t st) {
    if (lgc >= 3 && lgc <= 7) {   // fine 16^3 .. 256^3: rows staged in LDS
        const unsigned n = 2u << lgc;
        const unsigned blocks = (n / 2) * (n / kHoTy);
        const T h2 = (T)(h * h);
        const int R = order / 2;
        const size_t lds = (size_t)(kHoTy + 2 * R) * n * sizeof(T);
        if (order == 2) k_ho_resid_restrict_lds<1, T><<<blocks, kBlock, lds, st>>>(u, f, uc, uold, rc, lgc, h2);
        else if (order == 4) k_ho_resid_restrict_lds<2, T><<<blocks, kBlock, lds, st>>>(u, f, uc, uold, rc, lgc, h2);
        else k_ho_resid_restrict_lds<3, T><<<blocks, kBlock, lds, st>>>(u, f, uc, uold, rc, lgc, h2);
        return;
    }
    HO_DISPATCH(order, k_ho_resid_restrict, T, grid_for((size_t)1 << (3 * lgc)), u, f, uc, uold, rc, lgc,
                (T)(h * h));
}

template <class T>
void launch_ho_fas(const T* uc, T* fc, int lgc, double hc, int order, hipStream_t st) {
    HO_DISPATCH(order, k_ho_fas, T, grid_for((size_t)1 << (3 * lgc)), uc, fc, lgc, (T)(hc * hc));
}

template <class T>
void launch_ho_prolong(T* u, const T* uc, const T* uold, int lg, hipStream_t st) {
    k_ho_prolong<T><<<grid_for((size_t)1 << (3 * lg)), kBlock, 0, st>>>(u, uc, uold, lg);
}

template <class T>
void launch_ho_fill(T* a, int lg, T v, hipStream_t st) {
    const unsigned n = 1u << (3 * lg);
    k_ho_fill<T><<<grid_for(n), kBlock, 0, st>>>(a, n, v);
}

#define HO_INST(T)                                                                                          \
    template void launch_ho_half<T>(const T*, T*, const T*, int, double, int, int, hipStream_t, hipEvent_t,    \
                                    hipEvent_t);                                                            \
    template void launch_ho_resid_restrict<T>(const T*, const T*, T*, T*, T*, int, double, int, hipStream_t); \
    template void launch_ho_fas<T>(const T*, T*, int, double, int, hipStream_t);                              \
    template void launch_ho_prolong<T>(T*, const T*, const T*, int, hipStream_t);                             \
    template void launch_ho_fill<T>(T*, int, T, hipStream_t);
HO_INST(double)
HO_INST(float)

// The residual and its squared sum by the staged kernel on 16^3 .. 256^3 (n^2 / kHoTy <= kHoParts
// partial sums); false (nothing launched) on other sizes.
static_assert(256 * (256 / kHoTy) <= kHoParts, "one partial sum per staged tile at 256^3");
template <bool kR32>
static bool launch_ho_resid_lds(const double* u, const double* f, float* r32, int lg, double h2, int order,
                                double* part, double* out, hipStream_t st) {
    if (lg < 4 || lg > 8) return false;
    const unsigned n = 1u << lg;
    const unsigned blocks = n * (n / kHoTy);
    const int R = order / 2;
    const size_t lds = (size_t)(kHoTy + 2 * R) * n * sizeof(double);
    if (order == 2) k_ho_resid_lds<1, kR32><<<blocks, kBlock, lds, st>>>(u, f, r32, lg, h2, part);
    else if (order == 4) k_ho_resid_lds<2, kR32><<<blocks, kBlock, lds, st>>>(u, f, r32, lg, h2, part);
    else k_ho_resid_lds<3, kR32><<<blocks, kBlock, lds, st>>>(u, f, r32, lg, h2, part);
    k_ho_reduce<<<1, kBlock, 0, st>>>(part, (int)blocks, out);
    return true;
}

void launch_ho_resid32(const double* u, const double* f, float* r32, int lg, double h, int order, double* part,
                       double* out, hipStream_t st) {
    const double h2 = h * h;
    if (launch_ho_resid_lds<true>(u, f, r32, lg, h2, order, part, out, st)) return;
    const int nb = ho_parts(lg);
    if (order == 2) k_ho_resid32<1><<<nb, kBlock, 0, st>>>(u, f, r32, lg, h2, part);
    else if (order == 4) k_ho_resid32<2><<<nb, kBlock, 0, st>>>(u, f, r32, lg, h2, part);
    else k_ho_resid32<3><<<nb, kBlock, 0, st>>>(u, f, r32, lg, h2, part);
    k_ho_reduce<<<1, kBlock, 0, st>>>(part, nb, out);
}

void launch_ho_add32(double* u, const float* e, int lg, hipStream_t st) {
    k_ho_add32<<<grid_for((size_t)1 << (3 * lg)), kBlock, 0, st>>>(u, e, lg);
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
    const double h2 = h * h;
    if (launch_ho_resid_lds<false>(u, f, nullptr, lg, h2, order, part, out, st)) return;
    const int nb = ho_parts(lg);
    if (order == 2) k_ho_psum<1, 1><<<nb, kBlock, 0, st>>>(u, f, lg, h2, part);
    else if (order == 4) k_ho_psum<2, 1><<<nb, kBlock, 0, st>>>(u, f, lg, h2, part);
    else k_ho_psum<3, 1><<<nb, kBlock, 0, st>>>(u, f, lg, h2, part);
    k_ho_reduce<<<1, kBlock, 0, st>>>(part, nb, out);
}

// ----------------------------------------------------------------------------------------------
// Higher-order Laplacians on nested patches (Section 3.3 with Tables 1 and 2), natural order, FP64.
// A patch keeps R = order / 2 ghost layers per face (hoz_face_off), refreshed before each
// half-sweep and residual by k_hoz_ghost: for every fine column in front of a face, a polynomial
// of degree 2R through the 2R + 1 parent cells J - R .. J + R around its parent, along each
// transverse axis in turn (the first, then the second), for each of the R parent layers outside
// the face; then a polynomial of degree 2R normal to the face through those R values and the
// first R + 1 fine cells, at the R ghost centres; then the ghosts of the 2 x 2 columns in front of
// one parent face are shifted together so that the mean of their Table 2 fluxes equals the
// parent's flux through that face, whose covered cells are the live means of their children.
// ----------------------------------------------------------------------------------------------
namespace {

__device__ __forceinline__ size_t hoz_nat(const int* n, int x, int y, int z) {
    return ((size_t)x * n[1] + y) * n[2] + z;
}

// value at (x, y, z) of a patch, with at most one coordinate outside [0, n): inside from v,
// outside from the ghost layers
__device__ __forceinline__ double hoz_val(const double* __restrict__ v, const double* __restrict__ g, const int* n,
                                          int R, int x, int y, int z) {
    const int q[3] = {x, y, z};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (q[a] < 0 || q[a] >= n[a]) {
            const int side = q[a] >= n[a];
            const int layer = side ? q[a] - n[a] : -q[a] - 1;
            const int b = a == 0 ? 1 : 0, c = a == 2 ? 1 : 2;
            return g[hoz_face_off(n, R, 2 * a + side) + ((size_t)layer * n[b] + q[b]) * n[c] + q[c]];
        }
    }
    return v[hoz_nat(n, x, y, z)];
}

// sum_{s=1..R} w_s (((x-s) + (x+s)) + ((y-s) + (y+s))) + ((z-s) + (z+s))) on a patch with ghosts
template <int R>
__device__ __forceinline__ double hoz_off(const double* __restrict__ v, const double* __restrict__ g, const int* n,
                                          int x, int y, int z) {
    double acc = 0;
#pragma unroll
    for (int s = 1; s <= R; ++s) {
        const double px = hoz_val(v, g, n, R, x - s, y, z) + hoz_val(v, g, n, R, x + s, y, z);
        const double py = hoz_val(v, g, n, R, x, y - s, z) + hoz_val(v, g, n, R, x, y + s, z);
        const double pz = hoz_val(v, g, n, R, x, y, z - s) + hoz_val(v, g, n, R, x, y, z + s);
        acc += ho_w<R>(s) * ((px + py) + pz);
    }
    return acc;
}

// One block per row J of ghost groups of a face (blockIdx.y = face), 64 groups of 4 lanes per pass
// over the row.  The R outside parent layers that a pass's groups read - (2R + 1) rows around J by
// the pass's columns and R on either side - are staged in LDS once, instead of 4 (2R + 1)^2 R
// loads per group.  The parallel step is a tensor product: its sums along b (one per layer, fine
// row parity jb and staged column) go to LDS in a second stage, and each lane then takes 2R + 1
// of them along c, so every value is formed with the operations of the direct double sum.
// The parent's part of a ghost column - its R parallel values A and the R parent cells O in
// front of its group - does not change while the patch alone is smoothed: MODE 1 also stores it
// in part (2R doubles per face column, [column][m]), MODE 2 reads it from there and stages
// nothing.
template <int R, int MODE>
__global__ __launch_bounds__(kBlock) void k_hoz_ghost(const double* __restrict__ pu, const double* __restrict__ u,
                                                      double* __restrict__ g, double* __restrict__ part, HozPatch P,
                                                      HozW W, int flux_match) {
    constexpr int kG = kBlock / 4;            // groups per pass
    constexpr int kW = kG + 2 * R;            // staged columns
    constexpr int kIt = (R * (2 * R + 1) * kW + kBlock - 1) / kBlock;   // staging loads per lane
    __shared__ double S[R][2 * R + 1][kW];
    __shared__ double T[R][2][kW];            // T[k][jb][col] = sum_db par[jb][db] S[k][db][col]
    const int* n = P.n;
    const int face = (int)blockIdx.y;
    const int a = face >> 1, side = face & 1;
    const int b = a == 0 ? 1 : 0, c = a == 2 ? 1 : 2;
    const int J = (int)blockIdx.x;
    if (J >= n[b] / 2) return;                // rows of this face (the grid covers the longest)
    const int nc2 = n[c] / 2;
    const int tg = (int)threadIdx.x >> 2, q = (int)threadIdx.x & 3;
    const int jb = q >> 1, kc = q & 1;
    const int Jp = P.off[b] + J;
    auto parent = [&](int ia, int ib, int ic) {
        int qq[3];
        qq[a] = ia;
        qq[b] = ib;
        qq[c] = ic;
        if (P.pper)
            for (int k = 0; k < 3; ++k) qq[k] = qq[k] < 0 ? qq[k] + P.pn[k] : (qq[k] >= P.pn[k] ? qq[k] - P.pn[k] : qq[k]);
        return pu[hoz_nat(P.pn, qq[0], qq[1], qq[2])];
    };
    for (int K0 = 0; K0 < nc2; K0 += kG) {
        const int cnt = nc2 - K0 < kG ? nc2 - K0 : kG;
        const int Kp0 = P.off[c] + K0;
        const int ws = cnt + 2 * R;            // staged columns of this pass
        const int nst = R * (2 * R + 1) * ws;
        // every lane of a group takes part in the shuffles; lanes past the row repeat its last group
        const bool live = tg < cnt;
        const int Kl = live ? tg : cnt - 1;
        const int K = K0 + Kl;
        // all loads of the pass first: the staged parents, then the fine cells of the column
        // inwards from the face (layers 0 .. 2R - 1)
        double st[kIt];
#pragma unroll
        for (int it = 0; it < kIt; ++it) {
            const int i = (int)threadIdx.x + it * kBlock;
            st[it] = 0.0;
            if (MODE != 2 && i < nst) {
                const int col = i % ws, r = i / ws;
                const int db = r % (2 * R + 1), k = r / (2 * R + 1);
                const int on = side ? P.off[a] + n[a] / 2 + k : P.off[a] - 1 - k;
                st[it] = parent(on, Jp + db - R, Kp0 + col - R);
            }
        }
        double v[2 * R];
        if (MODE != 0 && a == 2) {
            // z faces of the workspace arrays (modes 1 and 2): the column's 2R cells are contiguous
            // in z and come as R 16-byte pairs (rows of even length)
            const double* col = u + hoz_nat(n, 2 * J + jb, 2 * K + kc, 0);
#pragma unroll
            for (int m = 0; m < R; ++m) {
                if (side) {
                    const double2 pr = *(const double2*)(col + (n[2] - 2 - 2 * m));
                    v[2 * m] = pr.y;
                    v[2 * m + 1] = pr.x;
                } else {
                    const double2 pr = *(const double2*)(col + 2 * m);
                    v[2 * m] = pr.x;
                    v[2 * m + 1] = pr.y;
                }
            }
        } else {
#pragma unroll
            for (int i = 0; i < 2 * R; ++i) {
                int p3[3];
                p3[a] = side ? n[a] - 1 - i : i;
                p3[b] = 2 * J + jb;
                p3[c] = 2 * K + kc;
                v[i] = u[hoz_nat(n, p3[0], p3[1], p3[2])];
            }
        }
        // this lane's column among the face's columns (the ghost layers' indexing); its part is
        // the 2R doubles A[0 .. R), O[0 .. R) at part + 2R ci, read and written as R pairs
        const size_t ci = hoz_face_off(n, 1, face) + (size_t)(2 * J + jb) * n[c] + (2 * K + kc);
        double* pc = part + 2 * R * ci;
        double A[R], O[R];
        if constexpr (MODE == 2) {
            double e[2 * R];
#pragma unroll
            for (int m = 0; m < R; ++m) {
                const double2 pr = *(const double2*)(pc + 2 * m);
                e[2 * m] = pr.x;
                e[2 * m + 1] = pr.y;
            }
#pragma unroll
            for (int k = 0; k < R; ++k) {
                A[k] = e[k];
                O[k] = e[R + k];
            }
        } else {
        if (K0) __syncthreads();              // the previous pass has read S and T
#pragma unroll
        for (int it = 0; it < kIt; ++it) {
            const int i = (int)threadIdx.x + it * kBlock;
            if (i < nst) {
                const int col = i % ws, r = i / ws;
                S[r / (2 * R + 1)][r % (2 * R + 1)][col] = st[it];
            }
        }
        __syncthreads();
        for (int i = (int)threadIdx.x; i < R * 2 * ws; i += (int)blockDim.x) {
            const int col = i % ws, r = i / ws, pj = r & 1, k = r >> 1;
            double ab = 0.0;
#pragma unroll
            for (int db = 0; db <= 2 * R; ++db) ab += W.par[pj][db] * S[k][db][col];
            T[k][pj][col] = ab;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < R; ++k) {
            double acc = 0.0;
#pragma unroll
            for (int dc = 0; dc <= 2 * R; ++dc) acc += W.par[kc][dc] * T[k][jb][Kl + dc];
            A[k] = acc;
            O[k] = S[k][R][Kl + R];
        }
        if (MODE == 1 && live) {
            double e[2 * R];
#pragma unroll
            for (int k = 0; k < R; ++k) {
                e[k] = A[k];
                e[R + k] = O[k];
            }
#pragma unroll
            for (int m = 0; m < R; ++m) *(double2*)(pc + 2 * m) = make_double2(e[2 * m], e[2 * m + 1]);
        }
        }
        double g0[R];
#pragma unroll
        for (int gl = 0; gl < R; ++gl) {
            double acc = 0.0;
#pragma unroll
            for (int m = 0; m < R; ++m) acc += W.nor[gl][m] * A[m];
#pragma unroll
            for (int i = 0; i <= R; ++i) acc += W.nor[gl][R + i] * v[i];
            g0[gl] = acc;
        }
        double delta = 0.0;
        if (flux_match) {
            const double h = P.h;
            double ff = 0.0;
#pragma unroll
            for (int m = 0; m < R; ++m) ff += W.F[m] * g0[R - 1 - m];
#pragma unroll
            for (int i = 0; i < R; ++i) ff += W.F[R + i] * v[i];
            ff /= h;
            const int base = (int)(threadIdx.x & 63) & ~3;
            auto mean4 = [&](double x) {
                const double x0 = __shfl(x, base, 64), x1 = __shfl(x, base + 1, 64);
                const double x2 = __shfl(x, base + 2, 64), x3 = __shfl(x, base + 3, 64);
                return ((x0 + x1) + (x2 + x3)) * 0.25;
            };
            const double mff = mean4(ff);
            double fc = 0.0;
#pragma unroll
            for (int m = 0; m < R; ++m) fc += W.F[m] * O[R - 1 - m];
#pragma unroll
            for (int k = 0; k < R; ++k) fc += W.F[R + k] * (0.5 * mean4(v[2 * k] + v[2 * k + 1]));
            fc /= 2.0 * h;
            delta = (fc - mff) * h / W.S;
        }
        if (live) {
            const size_t fo = hoz_face_off(n, R, face);
#pragma unroll
            for (int gl = 0; gl < R; ++gl)
                g[fo + ((size_t)gl * n[b] + (2 * J + jb)) * n[c] + (2 * K + kc)] = g0[gl] + delta;
        }
    }
}

// position t of an array of n[0] x n[1] x n[2] cells (fewer than 2^32) in natural order
__device__ __forceinline__ void hoz_decode(const int* n, size_t t, int& x, int& y, int& z) {
    const unsigned tt = (unsigned)t, n1 = (unsigned)n[1], n2 = (unsigned)n[2];
    const unsigned r = tt / n2;
    z = (int)(tt - r * n2);
    const unsigned xq = r / n1;
    y = (int)(r - xq * n1);
    x = (int)xq;
}

// One thread per pair of z-neighbours (z0, z0 + 1), z0 even: exactly one of them has the colour,
// so every lane computes one update; the pair is read and written as one 16-byte access (the
// patch arrays are workspace arrays, 256-byte aligned, with an even z extent).  Cells whose whole
// stencil lies inside the patch read their neighbours directly; the others through the ghost
// layers.  The sums have the order of hoz_off, so the bits do not depend on the path.
template <int R>
__global__ __launch_bounds__(kBlock) void k_hoz_half(const double* __restrict__ in, double* __restrict__ out,
                                                     const double* __restrict__ f, const double* __restrict__ g,
                                                     HozPatch P, double h2, int colour) {
    const unsigned n0 = (unsigned)P.n[0], n1 = (unsigned)P.n[1], n2 = (unsigned)P.n[2], n2h = n2 >> 1;
    const unsigned p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n0 * n1 * n2h) return;
    const unsigned row = p / n2h, zp = p - row * n2h;
    const unsigned x = row / n1, y = row - x * n1, z0 = 2 * zp;
    const unsigned q = (x + y + z0 + (unsigned)colour) & 1u;   // the pair's cell of the colour
    const unsigned z = z0 + q;
    const size_t t0 = (size_t)row * n2 + z0, t = t0 + q;
    const double2 cur = *(const double2*)(in + t0);
    double acc = 0;
    if (x >= (unsigned)R && x + R < n0 && y >= (unsigned)R && y + R < n1 && z >= (unsigned)R && z + R < n2) {
        const size_t sx = (size_t)n1 * n2;
#pragma unroll
        for (int s = 1; s <= R; ++s) {
            const double px = in[t - s * sx] + in[t + s * sx];
            const double py = in[t - (size_t)s * n2] + in[t + (size_t)s * n2];
            const double pz = in[t - s] + in[t + s];
            acc += ho_w<R>(s) * ((px + py) + pz);
        }
    } else {
        acc = hoz_off<R>(in, g, P.n, (int)x, (int)y, (int)z);
    }
    const double v = (h2 * f[t] - acc) / (3.0 * HoW<R>::w0);
    *(double2*)(out + t0) = q ? make_double2(cur.x, v) : make_double2(v, cur.y);
}

// Rows y0 - R .. y0 + ny + R - 1 of x plane x of a patch, with R cells on each side in z, into
// rows[(ny + 2R) x (n2 + 2R)]: the cells outside the patch from the ghost layers, the corners
// (which no stencil reads) zero.  The n2 cells of a row come as 16-byte pairs (from the patch, or
// from a y face's ghost layer; the arrays are workspace arrays with even rows), each thread's
// loads in batches of 4 before their LDS writes, so that they are in flight together; then the
// 2R z-halo cells of each row.
template <int R>
__device__ __forceinline__ void hoz_stage_rows(double* __restrict__ rows, const double* __restrict__ in,
                                               const double* __restrict__ g, const HozPatch& P, int x, int y0,
                                               int ny) {
    constexpr int kBatch = 4;
    const int n0 = P.n[0], n1 = P.n[1], n2 = P.n[2], n2h = n2 >> 1;
    const int W = n2 + 2 * R;
    const int nr = ny + 2 * R;
    const int np = nr * n2h;
    for (int i0 = (int)threadIdx.x; i0 < np; i0 += kBatch * (int)blockDim.x) {
        double2 v[kBatch];
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
            const int i = i0 + k * (int)blockDim.x;
            v[k] = make_double2(0.0, 0.0);
            if (i < np) {
                const int r = i / n2h, pz = i - r * n2h;
                const int y = y0 + r - R;
                const double* src;
                if (y >= 0 && y < n1) {
                    src = in + hoz_nat(P.n, x, y, 2 * pz);
                } else {
                    const int side = y >= n1, layer = side ? y - n1 : -y - 1;
                    src = g + hoz_face_off(P.n, R, 2 + side) + ((size_t)layer * n0 + x) * n2 + 2 * pz;
                }
                v[k] = *(const double2*)src;
            }
        }
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
            const int i = i0 + k * (int)blockDim.x;
            if (i < np) {
                const int r = i / n2h, pz = i - r * n2h;
                double* d = rows + r * W + R + 2 * pz;
                d[0] = v[k].x;
                d[1] = v[k].y;
            }
        }
    }
    for (int i = (int)threadIdx.x; i < nr * 2 * R; i += (int)blockDim.x) {
        const int r = i / (2 * R), k = i - r * (2 * R);
        const int y = y0 + r - R;
        const int cz = k < R ? k : n2 + k;     // z = cz - R: -R .. -1, or n2 .. n2 + R - 1
        double v = 0.0;
        if (y >= 0 && y < n1) v = hoz_val(in, g, P.n, R, x, y, cz - R);
        rows[r * W + cz] = v;
    }
}

// The same half-sweep with the y and z neighbours from LDS (as k_ho_half_lds on periodic levels):
// a block owns rows y0 .. y0 + kHoTy - 1 of one x plane and stages them with R rows on each side in
// y and R cells on each side in z, taking what lies outside the patch from the ghost layers (the
// corners, which no stencil reads, are zero); the 2R x-neighbours and f come from memory.  The
// sums have the order of hoz_off, so the bits are those of k_hoz_half.
template <int R>
__global__ __launch_bounds__(kBlock) void k_hoz_half_lds(const double* __restrict__ in, double* __restrict__ out,
                                                         const double* __restrict__ f, const double* __restrict__ g,
                                                         HozPatch P, double h2, int colour) {
    extern __shared__ __align__(16) unsigned char hz_smem[];
    double* rows = (double*)hz_smem;           // [kHoTy + 2R][n2 + 2R]
    const int n0 = P.n[0], n1 = P.n[1], n2 = P.n[2];
    const int W = n2 + 2 * R;
    const int tiles = (n1 + kHoTy - 1) / kHoTy;
    const int x = (int)blockIdx.x / tiles, y0 = ((int)blockIdx.x - x * tiles) * kHoTy;
    const int ny = n1 - y0 < kHoTy ? n1 - y0 : kHoTy;
    hoz_stage_rows<R>(rows, in, g, P, x, y0, ny);
    __syncthreads();
    const int n2h = n2 >> 1;
    const size_t sx = (size_t)n1 * n2;
    for (int t = (int)threadIdx.x; t < ny * n2h; t += (int)blockDim.x) {
        const int ry = t / n2h, zp = t - ry * n2h;
        const int y = y0 + ry, z0 = 2 * zp;
        const int q = (x + y + z0 + colour) & 1, z = z0 + q;
        const double* row = rows + (ry + R) * W + R;   // row[k] = value at (x, y, k)
        const size_t i0 = hoz_nat(P.n, x, y, z0), i = i0 + q;
        double acc = 0;
#pragma unroll
        for (int s = 1; s <= R; ++s) {
            const double xm = x - s >= 0 ? in[i - s * sx] : hoz_val(in, g, P.n, R, x - s, y, z);
            const double xp = x + s < n0 ? in[i + s * sx] : hoz_val(in, g, P.n, R, x + s, y, z);
            const double px = xm + xp;
            const double py = row[z - s * W] + row[z + s * W];
            const double pz = row[z - s] + row[z + s];
            acc += ho_w<R>(s) * ((px + py) + pz);
        }
        const double v = (h2 * f[i] - acc) / (3.0 * HoW<R>::w0);
        *(double2*)(out + i0) = q ? make_double2(row[z0], v) : make_double2(v, row[z0 + 1]);
    }
}

// Steps 3-5 on a patch with 8 lanes per coarse cell (lanes 8k .. 8k + 7 of a wave hold the
// children (a, b, e) in the order a, b, e): each lane forms one child's residual, reading its
// neighbours directly where the whole stencil lies inside the patch and through the ghost layers
// otherwise, all loads of a lane independent of each other; the first lane of the eight gathers
// the residuals and values by shuffles and sums them in the order (a, b, e).
template <int R>
__global__ __launch_bounds__(kBlock) void k_hoz_rr8(const double* __restrict__ u, const double* __restrict__ f,
                                                    const double* __restrict__ g, HozPatch P, double h2,
                                                    double* __restrict__ pu, double* __restrict__ pf,
                                                    double* __restrict__ uold) {
    const unsigned n0 = (unsigned)P.n[0], n1 = (unsigned)P.n[1], n2 = (unsigned)P.n[2];
    const unsigned c1 = n1 >> 1, c2 = n2 >> 1, nc = (n0 >> 1) * c1 * c2;
    const unsigned gt = blockIdx.x * blockDim.x + threadIdx.x;
    const unsigned l = gt & 7u;
    // lanes past the last coarse cell repeat it (every lane takes part in the shuffles)
    const bool live = (gt >> 3) < nc;
    const unsigned t = live ? gt >> 3 : nc - 1;
    const unsigned rw = t / c2, Z = t - rw * c2, X = rw / c1, Y = rw - X * c1;
    const unsigned x = 2 * X + (l >> 2), y = 2 * Y + ((l >> 1) & 1u), z = 2 * Z + (l & 1u);
    const size_t i = ((size_t)x * n1 + y) * n2 + z;
    const double uv = u[i];
    double off = 0;
    if (x >= (unsigned)R && x + R < n0 && y >= (unsigned)R && y + R < n1 && z >= (unsigned)R && z + R < n2) {
        const size_t sx = (size_t)n1 * n2;
#pragma unroll
        for (int s = 1; s <= R; ++s) {
            const double px = u[i - s * sx] + u[i + s * sx];
            const double py = u[i - (size_t)s * n2] + u[i + (size_t)s * n2];
            const double pz = u[i - s] + u[i + s];
            off += ho_w<R>(s) * ((px + py) + pz);
        }
    } else {
        off = hoz_off<R>(u, g, P.n, (int)x, (int)y, (int)z);
    }
    const double lap = (off + 3.0 * HoW<R>::w0 * uv) / h2;
    const double rr = f[i] - lap;
    const int base = (int)(threadIdx.x & 63) & ~7;
    double rs = 0.0, us = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        rs += __shfl(rr, base + k, 64);
        us += __shfl(uv, base + k, 64);
    }
    if (l != 0 || !live) return;
    const size_t pi = hoz_nat(P.pn, P.off[0] + (int)X, P.off[1] + (int)Y, P.off[2] + (int)Z);
    const double um = us * 0.125;
    pu[pi] = um;
    uold[t] = um;
    pf[pi] = rs * 0.125;
}

// Steps 3-5 on a patch with the y and z neighbours from LDS: a block owns coarse plane X and coarse
// rows Y0 .. Y0 + kHoTy / 2 - 1, stages both fine planes 2X and 2X + 1 over their kHoTy fine rows
// (hoz_stage_rows), and each thread takes one coarse cell, its 8 children in the order (a, b, e);
// the 2R x-neighbours and f come from memory.  The same values and sums as k_hoz_rr8.
template <int R>
__global__ __launch_bounds__(kBlock) void k_hoz_rr_lds(const double* __restrict__ u, const double* __restrict__ f,
                                                       const double* __restrict__ g, HozPatch P, double h2,
                                                       double* __restrict__ pu, double* __restrict__ pf,
                                                       double* __restrict__ uold) {
    extern __shared__ __align__(16) unsigned char hz_smem[];
    double* rows = (double*)hz_smem;           // [2][kHoTy + 2R][n2 + 2R]
    constexpr int kTc = kHoTy / 2;             // coarse rows per block
    const int n0 = P.n[0], n1 = P.n[1], n2 = P.n[2];
    const int c1 = n1 / 2, c2 = n2 / 2;
    const int W = n2 + 2 * R, PS = (kHoTy + 2 * R) * W;
    const int tiles = (c1 + kTc - 1) / kTc;
    const int X = (int)blockIdx.x / tiles, Y0 = ((int)blockIdx.x - X * tiles) * kTc;
    const int nyc = c1 - Y0 < kTc ? c1 - Y0 : kTc;
    hoz_stage_rows<R>(rows, u, g, P, 2 * X, 2 * Y0, 2 * nyc);
    hoz_stage_rows<R>(rows + PS, u, g, P, 2 * X + 1, 2 * Y0, 2 * nyc);
    __syncthreads();
    const size_t sx = (size_t)n1 * n2;
    const double w0x3 = 3.0 * HoW<R>::w0;
    for (int t = (int)threadIdx.x; t < nyc * c2; t += (int)blockDim.x) {
        const int ry = t / c2, Z = t - ry * c2, Y = Y0 + ry;
        double rs = 0.0, us = 0.0;
        // one (a, b) column at a time (its two children unrolled): all 8 at once needed 348 VGPRs
#pragma unroll 1
        for (int ab = 0; ab < 4; ++ab)
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const int a = ab >> 1, b = ab & 1;
                    const int x = 2 * X + a, y = 2 * Y + b, z = 2 * Z + e;
                    const double* row = rows + a * PS + (2 * ry + b + R) * W + R;   // row[k] = u(x, y, k)
                    const size_t i = hoz_nat(P.n, x, y, z);
                    const double uv = row[z];
                    double off = 0;
#pragma unroll
                    for (int s = 1; s <= R; ++s) {
                        const double xm = x - s >= 0 ? u[i - s * sx] : hoz_val(u, g, P.n, R, x - s, y, z);
                        const double xp = x + s < n0 ? u[i + s * sx] : hoz_val(u, g, P.n, R, x + s, y, z);
                        const double px = xm + xp;
                        const double py = row[z - s * W] + row[z + s * W];
                        const double pz = row[z - s] + row[z + s];
                        off += ho_w<R>(s) * ((px + py) + pz);
                    }
                    const double lap = (off + w0x3 * uv) / h2;
                    rs += f[i] - lap;
                    us += uv;
                }
        const size_t pi = hoz_nat(P.pn, P.off[0] + X, P.off[1] + Y, P.off[2] + Z);
        const double um = us * 0.125;
        pu[pi] = um;
        uold[((size_t)X * c1 + Y) * c2 + Z] = um;
        pf[pi] = rs * 0.125;
    }
}

// FAS right-hand side on the covered box: periodic power-of-two level (PER) or a patch interior
template <int R, bool PER>
__global__ __launch_bounds__(kBlock) void k_hoz_fas(const double* __restrict__ u, double* __restrict__ f, int n0,
                                                    int n1, int n2, int lo0, int lo1, int lo2, int c0, int c1, int c2,
                                                    double h2) {
    const int cn[3] = {c0, c1, c2}, n[3] = {n0, n1, n2};
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)c0 * c1 * c2) return;
    int X, Y, Z;
    hoz_decode(cn, t, X, Y, Z);
    const int x = lo0 + X, y = lo1 + Y, z = lo2 + Z;
    const size_t i = hoz_nat(n, x, y, z);
    double off;
    if constexpr (PER) {
        const int lg = __builtin_ctz((unsigned)n0);
        off = ho_off<R, double>(u, (unsigned)x, (unsigned)y, (unsigned)z, lg, (unsigned)n0 - 1);
    } else {
        off = hoz_off<R>(u, nullptr, n, x, y, z);   // the covered box keeps >= R cells from the faces
    }
    f[i] = f[i] + (off + 3.0 * HoW<R>::w0 * u[i]) / h2;
}

__global__ __launch_bounds__(kBlock) void k_hoz_prolong(double* __restrict__ u, HozPatch P,
                                                        const double* __restrict__ pu,
                                                        const double* __restrict__ uold) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)P.n[0] * P.n[1] * P.n[2]) return;
    int x, y, z;
    hoz_decode(P.n, t, x, y, z);
    const int cn[3] = {P.n[0] / 2, P.n[1] / 2, P.n[2] / 2};
    const int X = x >> 1, Y = y >> 1, Z = z >> 1;
    u[t] = u[t] + (pu[hoz_nat(P.pn, P.off[0] + X, P.off[1] + Y, P.off[2] + Z)] - uold[hoz_nat(cn, X, Y, Z)]);
}

__global__ __launch_bounds__(kBlock) void k_hoz_restrict(const double* __restrict__ v, HozPatch P,
                                                         double* __restrict__ pv) {
    const int cn[3] = {P.n[0] / 2, P.n[1] / 2, P.n[2] / 2};
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)cn[0] * cn[1] * cn[2]) return;
    int X, Y, Z;
    hoz_decode(cn, t, X, Y, Z);
    double s = 0.0;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int e = 0; e < 2; ++e) s += v[hoz_nat(P.n, 2 * X + a, 2 * Y + b, 2 * Z + e)];
    pv[hoz_nat(P.pn, P.off[0] + X, P.off[1] + Y, P.off[2] + Z)] = s * 0.125;
}

template <int R, int MODE>
__global__ __launch_bounds__(kBlock) void k_hoz_psum(const double* __restrict__ v, const double* __restrict__ f,
                                                     const double* __restrict__ g, int n0, int n1, int n2, int lo0,
                                                     int lo1, int lo2, int c0, int c1, int c2, double h2,
                                                     double* __restrict__ part) {
    const int n[3] = {n0, n1, n2};
    const size_t cells = (size_t)n0 * n1 * n2;
    double acc = 0.0;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < cells; t += (size_t)gridDim.x * blockDim.x) {
        int x, y, z;
        hoz_decode(n, t, x, y, z);
        if (x >= lo0 && x < lo0 + c0 && y >= lo1 && y < lo1 + c1 && z >= lo2 && z < lo2 + c2) continue;
        double val;
        if constexpr (MODE == 0) {
            val = v[t];
        } else if constexpr (MODE == 1) {
            val = f[t] - (hoz_off<R>(v, g, n, x, y, z) + 3.0 * HoW<R>::w0 * v[t]) / h2;
        } else {
            const int lg = __builtin_ctz((unsigned)n0);
            val = f[t] - (ho_off<R, double>(v, (unsigned)x, (unsigned)y, (unsigned)z, lg, (unsigned)n0 - 1) +
                          3.0 * HoW<R>::w0 * v[t]) / h2;
        }
        acc += val * val;
    }
    const double s = ho_block_sum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// MODE 1 of k_hoz_psum with the y and z neighbours from LDS: each block takes tiles of kHoTy rows
// of one x plane in turn (tile blockIdx.x, then + gridDim.x, ...) and stages them as
// k_hoz_half_lds does; every cell outside the covered box adds r^2, r = f - L u with the operations
// of hoz_off.  The partial sums run over other cells than in k_hoz_psum, so their last bits differ.
template <int R>
__global__ __launch_bounds__(kBlock) void k_hoz_psum_lds(const double* __restrict__ v, const double* __restrict__ f,
                                                         const double* __restrict__ g, HozPatch P, int lo0, int lo1,
                                                         int lo2, int c0, int c1, int c2, double h2,
                                                         double* __restrict__ part) {
    extern __shared__ __align__(16) unsigned char hz_smem[];
    double* rows = (double*)hz_smem;           // [kHoTy + 2R][n2 + 2R]
    const int n0 = P.n[0], n1 = P.n[1], n2 = P.n[2];
    const int W = n2 + 2 * R;
    const int tiles = (n1 + kHoTy - 1) / kHoTy;
    const size_t sx = (size_t)n1 * n2;
    const double w0x3 = 3.0 * HoW<R>::w0;
    double acc = 0.0;
    for (int tile = (int)blockIdx.x; tile < n0 * tiles; tile += (int)gridDim.x) {
        const int x = tile / tiles, y0 = (tile - x * tiles) * kHoTy;
        const int ny = n1 - y0 < kHoTy ? n1 - y0 : kHoTy;
        __syncthreads();                       // the previous tile has been read
        hoz_stage_rows<R>(rows, v, g, P, x, y0, ny);
        __syncthreads();
        const bool xcov = x >= lo0 && x < lo0 + c0;
        for (int t = (int)threadIdx.x; t < ny * n2; t += (int)blockDim.x) {
            const int ry = t / n2, z = t - ry * n2, y = y0 + ry;
            if (xcov && y >= lo1 && y < lo1 + c1 && z >= lo2 && z < lo2 + c2) continue;
            const double* row = rows + (ry + R) * W + R;
            const size_t i = hoz_nat(P.n, x, y, z);
            double off = 0;
#pragma unroll
            for (int s = 1; s <= R; ++s) {
                const double xm = x - s >= 0 ? v[i - s * sx] : hoz_val(v, g, P.n, R, x - s, y, z);
                const double xp = x + s < n0 ? v[i + s * sx] : hoz_val(v, g, P.n, R, x + s, y, z);
                const double px = xm + xp;
                const double py = row[z - s * W] + row[z + s * W];
                const double pz = row[z - s] + row[z + s];
                off += ho_w<R>(s) * ((px + py) + pz);
            }
            const double val = f[i] - (off + w0x3 * row[z]) / h2;
            acc += val * val;
        }
    }
    const double s = ho_block_sum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

}  // namespace

#define HOZ_R(order, STMT1, STMT2, STMT3) \
    do {                                  \
        if ((order) == 2) { STMT1; }      \
        else if ((order) == 4) { STMT2; } \
        else { STMT3; }                   \
    } while (0)

void launch_hoz_ghost(const double* pu, const double* u, double* g, const HozPatch& P, const HozW& W, int order,
                      int flux_match, hipStream_t st, double* part, int mode) {
    // one block per row of groups: n[b] / 2 rows on a face normal to a (b = 1 for a = 0, else 0)
    const dim3 grid((unsigned)std::max(P.n[1] / 2, P.n[0] / 2), 6);
    if (!part) mode = 0;
#define HOZ_GH(R)                                                                                    \
    do {                                                                                             \
        if (mode == 0) k_hoz_ghost<R, 0><<<grid, kBlock, 0, st>>>(pu, u, g, part, P, W, flux_match); \
        else if (mode == 1) k_hoz_ghost<R, 1><<<grid, kBlock, 0, st>>>(pu, u, g, part, P, W, flux_match); \
        else k_hoz_ghost<R, 2><<<grid, kBlock, 0, st>>>(pu, u, g, part, P, W, flux_match);        \
    } while (0)
    HOZ_R(order, HOZ_GH(1), HOZ_GH(2), HOZ_GH(3));
#undef HOZ_GH
}

void launch_hoz_half(const double* in, double* out, const double* f, const double* g, const HozPatch& P, int order,
                     int colour, hipStream_t st) {
    const double h2 = P.h * P.h;
    const int R = order / 2;
    const size_t lds = (size_t)(kHoTy + 2 * R) * (P.n[2] + 2 * R) * sizeof(double);
    if (lds <= 64u * 1024u) {   // rows staged in LDS (within the default limit: n_z up to 570)
        const unsigned grid = (unsigned)P.n[0] * (unsigned)((P.n[1] + kHoTy - 1) / kHoTy);
        HOZ_R(order, (k_hoz_half_lds<1><<<grid, kBlock, lds, st>>>(in, out, f, g, P, h2, colour)),
              (k_hoz_half_lds<2><<<grid, kBlock, lds, st>>>(in, out, f, g, P, h2, colour)),
              (k_hoz_half_lds<3><<<grid, kBlock, lds, st>>>(in, out, f, g, P, h2, colour)));
        return;
    }
    const int grid = grid_for((size_t)P.n[0] * P.n[1] * (P.n[2] / 2));   // pairs of z-neighbours
    HOZ_R(order, (k_hoz_half<1><<<grid, kBlock, 0, st>>>(in, out, f, g, P, h2, colour)),
          (k_hoz_half<2><<<grid, kBlock, 0, st>>>(in, out, f, g, P, h2, colour)),
          (k_hoz_half<3><<<grid, kBlock, 0, st>>>(in, out, f, g, P, h2, colour)));
}

void launch_hoz_resid_restrict(const double* u, const double* f, const double* g, const HozPatch& P, int order,
                               double* pu, double* pf, double* uold, hipStream_t st) {
    const double h2 = P.h * P.h;
    const int R = order / 2;
    const size_t lds = (size_t)2 * (kHoTy + 2 * R) * (P.n[2] + 2 * R) * sizeof(double);
    if (lds <= 64u * 1024u) {   // both fine planes of a coarse plane staged (n_z up to 280)
        const int tc = kHoTy / 2;
        const unsigned grid = (unsigned)(P.n[0] / 2) * (unsigned)((P.n[1] / 2 + tc - 1) / tc);
        HOZ_R(order, (k_hoz_rr_lds<1><<<grid, kBlock, lds, st>>>(u, f, g, P, h2, pu, pf, uold)),
              (k_hoz_rr_lds<2><<<grid, kBlock, lds, st>>>(u, f, g, P, h2, pu, pf, uold)),
              (k_hoz_rr_lds<3><<<grid, kBlock, lds, st>>>(u, f, g, P, h2, pu, pf, uold)));
        return;
    }
    const int grid = grid_for((size_t)8 * (P.n[0] / 2) * (P.n[1] / 2) * (P.n[2] / 2));   // 8 lanes per coarse cell
    HOZ_R(order, (k_hoz_rr8<1><<<grid, kBlock, 0, st>>>(u, f, g, P, h2, pu, pf, uold)),
          (k_hoz_rr8<2><<<grid, kBlock, 0, st>>>(u, f, g, P, h2, pu, pf, uold)),
          (k_hoz_rr8<3><<<grid, kBlock, 0, st>>>(u, f, g, P, h2, pu, pf, uold)));
}

void launch_hoz_fas(const double* u, double* f, const int* n, int periodic, const int* lo, const int* cn, double h,
                    int order, hipStream_t st) {
    const int grid = grid_for((size_t)cn[0] * cn[1] * cn[2]);
    const double h2 = h * h;
#define HOZ_FAS_ARGS u, f, n[0], n[1], n[2], lo[0], lo[1], lo[2], cn[0], cn[1], cn[2], h2
    if (periodic)
        HOZ_R(order, (k_hoz_fas<1, true><<<grid, kBlock, 0, st>>>(HOZ_FAS_ARGS)),
              (k_hoz_fas<2, true><<<grid, kBlock, 0, st>>>(HOZ_FAS_ARGS)),
              (k_hoz_fas<3, true><<<grid, kBlock, 0, st>>>(HOZ_FAS_ARGS)));
    else
        HOZ_R(order, (k_hoz_fas<1, false><<<grid, kBlock, 0, st>>>(HOZ_FAS_ARGS)),
              (k_hoz_fas<2, false><<<grid, kBlock, 0, st>>>(HOZ_FAS_ARGS)),
              (k_hoz_fas<3, false><<<grid, kBlock, 0, st>>>(HOZ_FAS_ARGS)));
#undef HOZ_FAS_ARGS
}

void launch_hoz_prolong(double* u, const HozPatch& P, const double* pu, const double* uold, hipStream_t st) {
    k_hoz_prolong<<<grid_for((size_t)P.n[0] * P.n[1] * P.n[2]), kBlock, 0, st>>>(u, P, pu, uold);
}

void launch_hoz_restrict(const double* v, const HozPatch& P, double* pv, hipStream_t st) {
    k_hoz_restrict<<<grid_for((size_t)(P.n[0] / 2) * (P.n[1] / 2) * (P.n[2] / 2)), kBlock, 0, st>>>(v, P, pv);
}

void launch_hoz_psum(int mode, const double* v, const double* f, const double* g, const int* n, const int* lo,
                     const int* cn, double h, int order, double* part, hipStream_t st) {
    const int nb = kHozParts;
    const double h2 = h * h;
#define HOZ_PS_ARGS v, f, g, n[0], n[1], n[2], lo[0], lo[1], lo[2], cn[0], cn[1], cn[2], h2, part
    const int R = order / 2;
    const size_t lds = (size_t)(kHoTy + 2 * R) * (n[2] + 2 * R) * sizeof(double);
    if (mode == 0) k_hoz_psum<1, 0><<<nb, kBlock, 0, st>>>(HOZ_PS_ARGS);
    else if (mode == 1 && lds <= 64u * 1024u) {
        HozPatch P{};
        for (int a = 0; a < 3; ++a) P.n[a] = n[a];
#define HOZ_PL_ARGS v, f, g, P, lo[0], lo[1], lo[2], cn[0], cn[1], cn[2], h2, part
        HOZ_R(order, (k_hoz_psum_lds<1><<<nb, kBlock, lds, st>>>(HOZ_PL_ARGS)),
              (k_hoz_psum_lds<2><<<nb, kBlock, lds, st>>>(HOZ_PL_ARGS)),
              (k_hoz_psum_lds<3><<<nb, kBlock, lds, st>>>(HOZ_PL_ARGS)));
#undef HOZ_PL_ARGS
    } else if (mode == 1)
        HOZ_R(order, (k_hoz_psum<1, 1><<<nb, kBlock, 0, st>>>(HOZ_PS_ARGS)),
              (k_hoz_psum<2, 1><<<nb, kBlock, 0, st>>>(HOZ_PS_ARGS)),
              (k_hoz_psum<3, 1><<<nb, kBlock, 0, st>>>(HOZ_PS_ARGS)));
    else
        HOZ_R(order, (k_hoz_psum<1, 2><<<nb, kBlock, 0, st>>>(HOZ_PS_ARGS)),
              (k_hoz_psum<2, 2><<<nb, kBlock, 0, st>>>(HOZ_PS_ARGS)),
              (k_hoz_psum<3, 2><<<nb, kBlock, 0, st>>>(HOZ_PS_ARGS)));
#undef HOZ_PS_ARGS
}

}  // namespace mgic
