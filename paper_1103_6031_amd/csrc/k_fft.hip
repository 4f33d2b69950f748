// Three-dimensional complex FFTs for gfx950 and the spectral multipliers of Section 3.5 (finite-
// volume and sub-grid deconvolution, the hybrid Poisson correction) and of the real-space
// transfer-function convolution of Section 2.2, fused into the transform's middle pass.
//
// A 3-D transform is three launches of batched 1-D transforms, one per axis.  A workgroup loads a
// tile of nl lines into LDS, zero-extending lines that are stored shorter than the transform (the
// zero padding of isolated boundaries is never materialised), runs a Stockham autosort FFT
// (radix 8, with one radix-2 or radix-4 stage first when log2 N is not a multiple of 3;
// Govindaraju et al. 2008, "High performance discrete Fourier transforms on graphics
// processors") with an LDS exchange between stages, and stores the first m_out points of each
// line.  Lines along z are contiguous in memory: the tile
// loads each line as one run.  Along y and x a tile holds nl lines that are consecutive in z, so
// every global access is a run of nl consecutive elements.  In LDS the tile is interleaved, point
// i of line l at i * (nl + 1) + l: lane-consecutive lines are address-consecutive during the
// stages, and the odd stride keeps the contiguous-line loads free of bank conflicts.  The N
// twiddles of the transform length follow the tile in LDS.
//
// The x pass can run forward, multiply every element by a multiplier of its (kx, ky, kz), and
// run the inverse in the same launch: the spectrum of the x pass never goes to memory.

#include "spec_internal.h"

namespace mgic {

namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

// radix-4 DFT in registers; forward uses e^{-2 pi i rk/4}, inverse e^{+2 pi i rk/4}
template <bool INV>
__device__ __forceinline__ void dft4(double2& a0, double2& a1, double2& a2, double2& a3) {
    const double2 s02 = cadd(a0, a2), d02 = csub(a0, a2);
    const double2 s13 = cadd(a1, a3), d13 = csub(a1, a3);
    // -i * d13 = (d13.y, -d13.x)
    const double2 mi = INV ? make_double2(-d13.y, d13.x) : make_double2(d13.y, -d13.x);
    a0 = cadd(s02, s13);
    a2 = csub(s02, s13);
    a1 = cadd(d02, mi);
    a3 = csub(d02, mi);
}

// radix-R DFT in registers (R = 2, 4, 8); the radix-8 one is two radix-4 DFTs of the even and odd
// points combined with the eighth roots of unity
template <int R, bool INV>
__device__ __forceinline__ void dft(double2* v) {
    if (R == 2) {
        const double2 a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if (R == 4) {
        dft4<INV>(v[0], v[1], v[2], v[3]);
    } else {
        double2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
        double2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
        dft4<INV>(e0, e1, e2, e3);
        dft4<INV>(o0, o1, o2, o3);
        const double r2 = 0.70710678118654752440;
        // w^k o_k, w = e^{-i pi / 4} (forward) or e^{+i pi / 4} (inverse)
        const double2 t1 = INV ? make_double2((o1.x - o1.y) * r2, (o1.x + o1.y) * r2)
                               : make_double2((o1.x + o1.y) * r2, (o1.y - o1.x) * r2);
        const double2 t2 = INV ? make_double2(-o2.y, o2.x) : make_double2(o2.y, -o2.x);
        const double2 t3 = INV ? make_double2((-o3.x - o3.y) * r2, (o3.x - o3.y) * r2)
                               : make_double2((o3.y - o3.x) * r2, (-o3.x - o3.y) * r2);
        v[0] = cadd(e0, o0);
        v[4] = csub(e0, o0);
        v[1] = cadd(e1, t1);
        v[5] = csub(e1, t1);
        v[2] = cadd(e2, t2);
        v[6] = csub(e2, t2);
        v[3] = cadd(e3, t3);
        v[7] = csub(e3, t3);
    }
}

// One Stockham stage on a tile of nl interleaved lines of length N = 2^lgN.  Butterfly j of a
// line reads points j + r N/R, twiddles them by w^(r k N / (Ns R)) with k = j mod Ns, and writes
// the radix-R DFT to points (j - k) R + k + r Ns.  twl holds e^{-2 pi i t / N}, t < N, in LDS.
template <int R, bool INV>
__device__ __forceinline__ void fft_stage(double2* lds, const double2* twl, int lgN, int lgnl, int lgNs) {
    constexpr int kIt = kFftTile / (R * kBlock);
    constexpr int lgR = R == 8 ? 3 : (R == 4 ? 2 : 1);
    const int nl = 1 << lgnl, LS = nl + 1;
    const int P = 1 << (lgN - lgR);
    const int items = nl * P;
    const int Ns = 1 << lgNs;
    const int tws = lgN - lgNs - lgR;   // k * N / (Ns R) = k << tws
    double2 v[kIt][R];
    int dst[kIt];
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
        const int q = (int)threadIdx.x + it * kBlock;
        if (q < items) {
            const int l = q & (nl - 1), j = q >> lgnl;
            const int k = j & (Ns - 1);
#pragma unroll
            for (int r = 0; r < R; ++r) v[it][r] = lds[(j + r * P) * LS + l];
            const int step = k << tws;
#pragma unroll
            for (int r = 1; r < R; ++r) {
                double2 w = twl[r * step];
                if (INV) w.y = -w.y;
                v[it][r] = cmul(v[it][r], w);
            }
            dft<R, INV>(v[it]);
            dst[it] = ((j - k) << lgR) + k;
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
        const int q = (int)threadIdx.x + it * kBlock;
        if (q < items) {
            const int l = q & (nl - 1);
#pragma unroll
            for (int r = 0; r < R; ++r) lds[(dst[it] + r * Ns) * LS + l] = v[it][r];
        }
    }
    __syncthreads();
}

template <bool INV>
__device__ __forceinline__ void fft_tile(double2* lds, const double2* twl, int lgN, int lgnl) {
    int lgNs = 0;
    const int rem = lgN % 3;
    if (rem == 1) {
        fft_stage<2, INV>(lds, twl, lgN, lgnl, 0);
        lgNs = 1;
    } else if (rem == 2) {
        fft_stage<4, INV>(lds, twl, lgN, lgnl, 0);
        lgNs = 2;
    }
    for (; lgNs < lgN; lgNs += 3) fft_stage<8, INV>(lds, twl, lgN, lgnl, lgNs);
}

template <int IN>
__device__ __forceinline__ double2 load_in(const FftPass& A, long long idx) {
    if (IN == kFftInCplx) return ((const double2*)A.in0)[idx];
    if (IN == kFftInRe) return make_double2(((const double*)A.in0)[idx], 0.0);
    return make_double2(((const double*)A.in0)[idx], ((const double*)A.in1)[idx]);
}

template <int OUT>
__device__ __forceinline__ void store_out(const FftPass& A, long long idx, double2 v) {
    if (OUT == kFftOutCplx) {
        ((double2*)A.out0)[idx] = v;
    } else if (OUT == kFftOutRe) {
        ((double*)A.out0)[idx] = v.x;
    } else if (OUT == kFftOutRePairStore) {
        ((double*)A.out0)[idx] = v.x;
        if (A.out1) ((double*)A.out1)[idx] = v.y;
    } else {   // kFftOutRePairAdd
        double* o0 = (double*)A.out0;
        o0[idx] = o0[idx] + v.x;
        if (A.out1) {
            double* o1 = (double*)A.out1;
            o1[idx] = o1[idx] + v.y;
        }
    }
}

// the multiplier of spectral element (kx, ky, kz) = (i, a, b), applied to v
template <int SYM>
__device__ __forceinline__ double2 apply_sym(const FftPass& A, int i, int a, int b, double2 v) {
    const double c = A.sym_scale;
    if (SYM == kSymSeparable) {
        const double m = ((A.tab_x[i] * A.tab_y[a]) * A.tab_z[b]) * c;
        return make_double2(v.x * m, v.y * m);
    }
    if (SYM == kSymTable) {
        const double m = A.tab[(long long)i * A.tab_si + (long long)a * A.tab_sa + b] * c;
        return make_double2(v.x * m, v.y * m);
    }
    if (SYM == kSymInvLap) {
        // 1 / lambda(k), lambda = sum_axes of the per-axis Laplacian symbol; the k = 0 mode -> 0
        const double lam = (A.tab_x[i] + A.tab_y[a]) + A.tab_z[b];
        if (i == 0 && a == 0 && b == 0) return make_double2(0.0, 0.0);
        const double m = c / lam;
        return make_double2(v.x * m, v.y * m);
    }
    if (SYM == kSymReplace) {
        // modes below the coarse grid's Nyquist on every axis take 8 C(m) prod_a e^{-i pi m_a / P_a}
        // (per-axis phase tables hold cos, sin pairs); the rest keep the fine spectrum
        const int px = A.sym_n[0], py = A.sym_n[1], pz = A.sym_n[2];
        const int mx = i < px / 2 ? i : i - px, my = a < py / 2 ? a : a - py, mz = b < pz / 2 ? b : b - pz;
        const int cx = A.cn[0], cy = A.cn[1], cz = A.cn[2];
        if (2 * abs(mx) < cx && 2 * abs(my) < cy && 2 * abs(mz) < cz) {
            const int ix = mx < 0 ? mx + cx : mx, iy = my < 0 ? my + cy : my, iz = mz < 0 ? mz + cz : mz;
            const double2 C = A.csp[((long long)ix * cy + iy) * cz + iz];
            double2 w = make_double2(8.0 * C.x, 8.0 * C.y);
            w = cmul(w, make_double2(A.tab_x[2 * i], A.tab_x[2 * i + 1]));
            w = cmul(w, make_double2(A.tab_y[2 * a], A.tab_y[2 * a + 1]));
            w = cmul(w, make_double2(A.tab_z[2 * b], A.tab_z[2 * b + 1]));
            v = w;
        }
        return make_double2(v.x * c, v.y * c);
    }
    // hybrid correction: per-axis blocks [k^2 | lambda_1d | k (0 on Nyquist) | g (0 on Nyquist)]
    const double* X = A.tab_x;
    const double* Y = A.tab_y;
    const double* Z = A.tab_z;
    const int px = A.sym_n[0], py = A.sym_n[1], pz = A.sym_n[2];
    const double k2 = (X[i] + Y[a]) + Z[b];
    if (k2 == 0.0) return make_double2(0.0, 0.0);
    const double lam = (X[px + i] + Y[py + a]) + Z[pz + b];
    if (SYM == kSymHybridXY) {
        // components x and y packed as one complex field: (i s_x - s_y) f~
        const double sx = -X[2 * px + i] / k2 - X[3 * px + i] / lam;
        const double sy = -Y[2 * py + a] / k2 - Y[3 * py + a] / lam;
        return cmul(v, make_double2(-sy * c, sx * c));
    }
    const double sz = -Z[2 * pz + b] / k2 - Z[3 * pz + b] / lam;
    return cmul(v, make_double2(0.0, sz * c));
}

// One pass of 1-D transforms of length N = 2^lgN over the lines (a, b) of a 3-D array.
// CONTIG: lines are contiguous (si = 1), a tile is nl consecutive a (b unused).
// Otherwise: a tile is one a and nl consecutive b (sb = 1).
// Tile point e (of nl N) is line e >> lgN, point e & (N - 1) (CONTIG), or line e & (nl - 1), point
// e >> lgnl: consecutive lanes touch consecutive global addresses either way.  Every lane issues
// all of its loads before it writes any of them to LDS.
template <bool CONTIG>
__device__ __forceinline__ void tile_coords(int e, int lgN, int lgnl, int& l, int& i) {
    if (CONTIG) {
        l = e >> lgN;
        i = e & ((1 << lgN) - 1);
    } else {
        l = e & ((1 << lgnl) - 1);
        i = e >> lgnl;
    }
}

template <bool CONTIG, int IN, int OUT, int OP, int SYM>
__global__ __launch_bounds__(kBlock) void k_fft_pass(FftPass A) {
    extern __shared__ __align__(16) unsigned char fft_smem[];
    constexpr int kLd = kFftTile / kBlock;
    const int lgnl = A.lgnl, nl = 1 << lgnl, LS = nl + 1, lgN = A.lgN, N = 1 << lgN;
    double2* lds = (double2*)fft_smem;
    double2* twl = lds + N * LS;
    int a, b0;
    if (CONTIG) {
        a = (int)blockIdx.x << lgnl;
        b0 = 0;
    } else {
        const int nbt = (A.nb + nl - 1) >> lgnl;
        a = (int)blockIdx.x / nbt;
        b0 = ((int)blockIdx.x - a * nbt) << lgnl;
    }
    const int total = nl << lgN;
    // load (zero beyond m_in and for lines past the end), with this length's twiddles
    {
        double2 r[kLd];
#pragma unroll
        for (int k = 0; k < kLd; ++k) {
            const int e = (int)threadIdx.x + k * kBlock;
            r[k] = make_double2(0.0, 0.0);
            if (e < total) {
                int l, i;
                tile_coords<CONTIG>(e, lgN, lgnl, l, i);
                if (CONTIG) {
                    if (a + l < A.na && i < A.m_in) r[k] = load_in<IN>(A, (long long)(a + l) * A.in_sa + i);
                } else {
                    if (b0 + l < A.nb && i < A.m_in)
                        r[k] = load_in<IN>(A, (long long)a * A.in_sa + b0 + l + (long long)i * A.in_si);
                }
            }
        }
        for (int t = (int)threadIdx.x; t < N; t += kBlock) twl[t] = A.tw[t << (A.lgtw - lgN)];
#pragma unroll
        for (int k = 0; k < kLd; ++k) {
            const int e = (int)threadIdx.x + k * kBlock;
            if (e < total) {
                int l, i;
                tile_coords<CONTIG>(e, lgN, lgnl, l, i);
                lds[i * LS + l] = r[k];
            }
        }
    }
    __syncthreads();
    if (OP == kFftInverse) {
        fft_tile<true>(lds, twl, lgN, lgnl);
    } else {
        fft_tile<false>(lds, twl, lgN, lgnl);
        if (OP == kFftFwdSymInv) {
#pragma unroll
            for (int k = 0; k < kLd; ++k) {
                const int e = (int)threadIdx.x + k * kBlock;
                if (e < total) {
                    const int l = e & (nl - 1), i = e >> lgnl;
                    if (b0 + l < A.nb) lds[i * LS + l] = apply_sym<SYM>(A, i, a, b0 + l, lds[i * LS + l]);
                }
            }
            __syncthreads();
            fft_tile<true>(lds, twl, lgN, lgnl);
        }
    }
    // store the first m_out points of every line
#pragma unroll
    for (int k = 0; k < kLd; ++k) {
        const int e = (int)threadIdx.x + k * kBlock;
        if (e < total) {
            int l, i;
            tile_coords<CONTIG>(e, lgN, lgnl, l, i);
            if (i < A.m_out) {
                if (CONTIG) {
                    if (a + l < A.na) store_out<OUT>(A, (long long)(a + l) * A.out_sa + i, lds[i * LS + l]);
                } else {
                    if (b0 + l < A.nb)
                        store_out<OUT>(A, (long long)a * A.out_sa + b0 + l + (long long)i * A.out_si, lds[i * LS + l]);
                }
            }
        }
    }
}

// e^{-2 pi i t / 2^lg} for t < 2^lg
__global__ void k_fft_twiddles(double2* tw, int lg) {
    const int t = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (t >= (1 << lg)) return;
    double s, c;
    sincospi(2.0 * (double)t / (double)(1 << lg), &s, &c);
    tw[t] = make_double2(c, -s);
}

// Per-axis multiplier tables.  Mode m of an axis of P points (m = t for t < P/2, t - P above) has
// kh = 2 pi m / P.  kind kSymFv: 1 / sinc(kh/2); kSymSg: 1 / cos(kh/4); hybrid: the four blocks
// [kh^2 | Laplacian symbol of the order | kh, 0 on Nyquist | gradient symbol g, 0 on Nyquist].
__global__ void k_spec_tables(double* t0, double* t1, double* t2, int p0, int p1, int p2, int kind, int lap_order,
                              int grad_order) {
    int t = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    double* tab;
    int P;
    if (t < p0) {
        tab = t0;
        P = p0;
    } else if (t < p0 + p1) {
        tab = t1;
        P = p1;
        t -= p0;
    } else if (t < p0 + p1 + p2) {
        tab = t2;
        P = p2;
        t -= p0 + p1;
    } else {
        return;
    }
    const int m = t < P / 2 ? t : t - P;
    const double q = 2.0 * (double)m / (double)P;   // kh / pi
    const double kh = 3.14159265358979323846 * q;
    if (kind == kSpecFv) {
        double s, c;
        sincospi(0.5 * q, &s, &c);
        tab[t] = m == 0 ? 1.0 : (0.5 * kh) / s;
        return;
    }
    if (kind == kSpecSg) {
        tab[t] = 1.0 / cospi(0.25 * q);
        return;
    }
    if (kind == kSpecPoisson) {   // the 1-D Laplacian symbol of the order, in grid units
        double s1, c1, s2, c2, s3, c3;
        sincospi(q, &s1, &c1);
        sincospi(2.0 * q, &s2, &c2);
        sincospi(3.0 * q, &s3, &c3);
        if (lap_order == 2) tab[t] = -2.0 * (1.0 - c1);
        else if (lap_order == 4) tab[t] = -(c2 - 16.0 * c1 + 15.0) / 6.0;
        else tab[t] = -(-2.0 * c3 + 27.0 * c2 - 270.0 * c1 + 245.0) / 90.0;
        return;
    }
    if (kind == kSpecReplace) {   // e^{-i pi m / P}: the fine centres sit a quarter coarse cell off
        double s, c;
        sincospi((double)m / (double)P, &s, &c);
        tab[2 * t] = c;
        tab[2 * t + 1] = -s;
        return;
    }
    double s1, c1, s2, c2, s3, c3;
    sincospi(q, &s1, &c1);
    sincospi(2.0 * q, &s2, &c2);
    sincospi(3.0 * q, &s3, &c3);
    double lam;
    if (lap_order == 2) lam = -2.0 * (1.0 - c1);
    else if (lap_order == 4) lam = -(c2 - 16.0 * c1 + 15.0) / 6.0;
    else lam = -(-2.0 * c3 + 27.0 * c2 - 270.0 * c1 + 245.0) / 90.0;
    double g;
    if (grad_order == 4) g = (8.0 * s1 - s2) / 6.0;
    else g = (45.0 * s1 - 9.0 * s2 + s3) / 30.0;
    const bool nyq = 2 * t == P;
    tab[t] = kh * kh;
    tab[P + t] = lam;
    tab[2 * P + t] = nyq ? 0.0 : kh;
    tab[3 * P + t] = nyq ? 0.0 : g;
}

template <bool CONTIG, int IN, int OUT, int OP, int SYM>
hipError_t run_pass(const FftPass& A, hipStream_t st) {
    const int nl = 1 << A.lgnl;
    const unsigned lds = (unsigned)((1u << A.lgN) * (unsigned)(nl + 2) * sizeof(double2));
    const void* fn = (const void*)k_fft_pass<CONTIG, IN, OUT, OP, SYM>;
    static bool raised = false;
    if (!raised) {
        const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kFftMaxLds);
        if (e != hipSuccess) return e;
        raised = true;
    }
    unsigned blocks;
    if (CONTIG) blocks = (unsigned)((A.na + nl - 1) / nl);
    else blocks = (unsigned)A.na * (unsigned)((A.nb + nl - 1) / nl);
    if (blocks == 0) return hipSuccess;
    k_fft_pass<CONTIG, IN, OUT, OP, SYM><<<blocks, kBlock, lds, st>>>(A);
    return hipGetLastError();
}

}  // namespace

int fft_lines_per_tile(int lgN) {   // log2 of the tile's line count: nl * N <= kFftTile, nl <= 16
    int lg = 4;
    while (lg > 0 && (1 << (lg + lgN)) > kFftTile) --lg;
    return lg;
}

hipError_t launch_fft_twiddles(double2* tw, int lg, hipStream_t st) {
    k_fft_twiddles<<<((1 << lg) + kBlock - 1) / kBlock, kBlock, 0, st>>>(tw, lg);
    return hipGetLastError();
}

hipError_t launch_spec_tables(double* t0, double* t1, double* t2, const int P[3], int kind, int lap_order,
                              int grad_order, hipStream_t st) {
    const int total = P[0] + P[1] + P[2];
    k_spec_tables<<<(total + kBlock - 1) / kBlock, kBlock, 0, st>>>(t0, t1, t2, P[0], P[1], P[2], kind, lap_order,
                                                                     grad_order);
    return hipGetLastError();
}

// dispatch on the combinations the host pipelines use
hipError_t launch_fft_pass(const FftPass& A, bool contig, int in, int out, int op, int sym, hipStream_t st) {
    if (contig) {
        if (op == kFftForward && in == kFftInRe && out == kFftOutCplx)
            return run_pass<true, kFftInRe, kFftOutCplx, kFftForward, 0>(A, st);
        if (op == kFftForward && in == kFftInRePair && out == kFftOutCplx)
            return run_pass<true, kFftInRePair, kFftOutCplx, kFftForward, 0>(A, st);
        if (op == kFftForward && in == kFftInCplx && out == kFftOutCplx)
            return run_pass<true, kFftInCplx, kFftOutCplx, kFftForward, 0>(A, st);
        if (op == kFftInverse && in == kFftInCplx && out == kFftOutRePairStore)
            return run_pass<true, kFftInCplx, kFftOutRePairStore, kFftInverse, 0>(A, st);
        if (op == kFftInverse && in == kFftInCplx && out == kFftOutRePairAdd)
            return run_pass<true, kFftInCplx, kFftOutRePairAdd, kFftInverse, 0>(A, st);
        if (op == kFftInverse && in == kFftInCplx && out == kFftOutCplx)
            return run_pass<true, kFftInCplx, kFftOutCplx, kFftInverse, 0>(A, st);
        return hipErrorInvalidValue;
    }
    if (in != kFftInCplx) return hipErrorInvalidValue;
    if (op == kFftForward && out == kFftOutCplx) return run_pass<false, kFftInCplx, kFftOutCplx, kFftForward, 0>(A, st);
    if (op == kFftForward && out == kFftOutRe) return run_pass<false, kFftInCplx, kFftOutRe, kFftForward, 0>(A, st);
    if (op == kFftInverse && out == kFftOutCplx) return run_pass<false, kFftInCplx, kFftOutCplx, kFftInverse, 0>(A, st);
    if (op == kFftFwdSymInv && out == kFftOutCplx) {
        switch (sym) {
            case kSymSeparable: return run_pass<false, kFftInCplx, kFftOutCplx, kFftFwdSymInv, kSymSeparable>(A, st);
            case kSymTable: return run_pass<false, kFftInCplx, kFftOutCplx, kFftFwdSymInv, kSymTable>(A, st);
            case kSymHybridXY: return run_pass<false, kFftInCplx, kFftOutCplx, kFftFwdSymInv, kSymHybridXY>(A, st);
            case kSymHybridZ: return run_pass<false, kFftInCplx, kFftOutCplx, kFftFwdSymInv, kSymHybridZ>(A, st);
            case kSymReplace: return run_pass<false, kFftInCplx, kFftOutCplx, kFftFwdSymInv, kSymReplace>(A, st);
            case kSymInvLap: return run_pass<false, kFftInCplx, kFftOutCplx, kFftFwdSymInv, kSymInvLap>(A, st);
            default: return hipErrorInvalidValue;
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace mgic
