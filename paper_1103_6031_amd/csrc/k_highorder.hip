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

// steps 3-5 for one coarse cell: the mean of the 8 children's residuals and of their values
template <int R, class T>
__global__ __launch_bounds__(kBlock) void k_ho_resid_restrict(const T* __restrict__ u, const T* __restrict__ f,
                                                              T* __restrict__ uc, T* __restrict__ uold,
                                                              T* __restrict__ rc, int lgc, T h2) {
    const unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
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
    if (MODE == 0) {
        for (unsigned t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) acc += a[t];
    } else {   // pairs of z-neighbours (n is even)
        for (unsigned p = blockIdx.x * blockDim.x + threadIdx.x; p < n / 2; p += gridDim.x * blockDim.x) {
            const unsigned t = 2 * p, z = t & m, y = (t >> lg) & m, x = t >> (2 * lg);
            double2 uv;
            const double2 r = ho_pair_resid<R, double>(a, f, x, y, z, lg, m, h2, &uv);
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

// mixed precision: r32 = (float)(f - L u) in FP64, with the partial sums of r^2 (pairs of cells)
template <int R>
__global__ __launch_bounds__(kBlock) void k_ho_resid32(const double* __restrict__ u, const double* __restrict__ f,
                                                       float* __restrict__ r32, int lg, double h2,
                                                       double* __restrict__ part) {
    const unsigned n = 1u << (3 * lg), m = (1u << lg) - 1;
    double acc = 0.0;
    for (unsigned p = blockIdx.x * blockDim.x + threadIdx.x; p < n / 2; p += gridDim.x * blockDim.x) {
        const unsigned t = 2 * p, z = t & m, y = (t >> lg) & m, x = t >> (2 * lg);
        double2 uv;
        const double2 r = ho_pair_resid<R, double>(u, f, x, y, z, lg, m, h2, &uv);
        *(float2*)(r32 + t) = make_float2((float)r.x, (float)r.y);
        acc += r.x * r.x;
        acc += r.y * r.y;
    }
    const double s = ho_block_sum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
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
    const int g = grid_for((size_t)1 << (3 * lg - 1));   // pairs of cells (lg >= 1)
    if (ea) (void)hipEventRecord(ea, st);
    HO_DISPATCH(order, k_ho_half, T, g, in, out, f, lg, (T)(h * h), colour);
    if (eb) (void)hipEventRecord(eb, st);
}

template <class T>
void launch_ho_resid_restrict(const T* u, const T* f, T* uc, T* uold, T* rc, int lgc, double h, int order,
                              hipStream_t st) {
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

void launch_ho_resid32(const double* u, const double* f, float* r32, int lg, double h, int order, double* part,
                       double* out, hipStream_t st) {
    const int nb = ho_parts(lg);
    const double h2 = h * h;
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
    const int nb = ho_parts(lg);
    const double h2 = h * h;
    if (order == 2) k_ho_psum<1, 1><<<nb, kBlock, 0, st>>>(u, f, lg, h2, part);
    else if (order == 4) k_ho_psum<2, 1><<<nb, kBlock, 0, st>>>(u, f, lg, h2, part);
    else k_ho_psum<3, 1><<<nb, kBlock, 0, st>>>(u, f, lg, h2, part);
    k_ho_reduce<<<1, kBlock, 0, st>>>(part, nb, out);
}

}  // namespace mgic
