// Internal declarations of the spectral side of the library: the three-pass FFT (k_fft.hip), its
// host pipelines (spectral.cpp) and the multi-scale density (k_density.hip, density.cpp).
// Not part of the public ABI (see include/mgic.h).
#pragma once

#include "mg_internal.h"

namespace mgic {

// ---- three-dimensional FFTs (k_fft.hip) -------------------------------------------------------
constexpr int kFftTile = 2048;                       // complex points per workgroup tile
constexpr int kFftMaxLgN = 10;                       // transforms of length 2 .. 1024
constexpr unsigned kFftMaxLds = 1024u * 4u * 16u;    // N (nl + 2) 16 B, largest at N = 1024, nl = 2
enum { kFftInCplx = 0, kFftInRe = 1, kFftInRePair = 2 };
enum { kFftOutCplx = 0, kFftOutRe = 1, kFftOutRePairStore = 2, kFftOutRePairAdd = 3 };
enum { kFftForward = 0, kFftInverse = 1, kFftFwdSymInv = 2 };
enum { kSymSeparable = 1, kSymTable = 2, kSymHybridXY = 3, kSymHybridZ = 4, kSymReplace = 5, kSymInvLap = 6 };
enum { kSpecFv = 1, kSpecSg = 2, kSpecHybrid = 3, kSpecReplace = 4, kSpecPoisson = 5 };
// one pass of batched 1-D transforms: line (a, b) holds point i at a*sa + b + i*si (strided
// passes) or a*sa + i (contiguous passes); the input line has m_in points (the rest is zero),
// the first m_out points of the output line are stored
struct FftPass {
    int lgN = 0, lgnl = 0, lgtw = 0;
    int m_in = 0, m_out = 0;
    int na = 0, nb = 1;
    long long in_sa = 0, in_si = 1, out_sa = 0, out_si = 1;
    const void* in0 = nullptr;
    const void* in1 = nullptr;
    void* out0 = nullptr;
    void* out1 = nullptr;
    const double2* tw = nullptr;
    // multiplier of the fused x pass: element (kx, ky, kz) = (point, a, b)
    const double* tab_x = nullptr;
    const double* tab_y = nullptr;
    const double* tab_z = nullptr;
    int sym_n[3] = {0, 0, 0};
    const double* tab = nullptr;
    long long tab_si = 0, tab_sa = 0;
    const double2* csp = nullptr;   // kSymReplace: the coarse region's spectrum, cn[0] x cn[1] x cn[2]
    int cn[3] = {0, 0, 0};
    double sym_scale = 1.0;
};
int fft_lines_per_tile(int lgN);
hipError_t launch_fft_twiddles(double2* tw, int lg, hipStream_t st);
hipError_t launch_spec_tables(double* t0, double* t1, double* t2, const int P[3], int kind, int lap_order,
                              int grad_order, hipStream_t st);
hipError_t launch_fft_pass(const FftPass& A, bool contig, int in, int out, int op, int sym, hipStream_t st);
// a 3-D transform grid: a field of n cells per axis transformed on P points per axis (P = n
// periodic, the zero-padded isolated length otherwise), with its twiddles, multiplier tables and
// the work arrays W1 [n0][n1][P2], W2 = W3 [n0][P1][P2] (complex)
struct SpecGrid {
    int n[3] = {0, 0, 0};
    int P[3] = {0, 0, 0};
    int lg[3] = {0, 0, 0};
    int lgtw = 0;
    double2* tw = nullptr;
    double* tab[3] = {nullptr, nullptr, nullptr};
    double2* W1 = nullptr;
    double2* W2 = nullptr;
    double2* W3 = nullptr;
};
int spec_grid_init(const int* n, int isolated, SpecGrid& S);
void spec_grid_carve(SpecGrid& S, char* base, size_t& off);           // twiddles and tables
void spec_grid_work(const SpecGrid& S, size_t& w1, size_t& w2);       // complex points of W1, W2 (= W3)
hipError_t spec_grid_prepare(const SpecGrid& S, int kind, int lap_order, int grad_order, hipStream_t st);
hipError_t spec_forward_zy(const SpecGrid& S, const double* in0, const double* in1, hipStream_t st);
hipError_t spec_x_pass(const SpecGrid& S, int op, int out_kind, int sym, double scale, const double* tab,
                       const double2* csp, const int* cn, void* out, hipStream_t st);
hipError_t spec_inverse_yz(const SpecGrid& S, double* out0, double* out1, bool add, hipStream_t st);
// ---- multi-scale density (k_density.hip) -------------------------------------------------------
// a box of cells of a parent array: array dims pd, the parent's own cells start at po inside the
// array, the box starts at lo in the parent's own cells; wrap > 0: periodic with wrap cells per axis
struct DensBox {
    int pd[3] = {0, 0, 0};
    int po[3] = {0, 0, 0};
    int lo[3] = {0, 0, 0};
    int wrap = 0;
};
hipError_t launch_kernel_direct(double* T, const int* P, double h, const double* table, double dr, int subgrid,
                                hipStream_t st);
hipError_t launch_kernel_restrict(double* Tc, const int* P, double h, const double* Tf, const int* Pf,
                                  const double* table, double dr, hipStream_t st);
hipError_t launch_divide(double* out, const double* in, size_t n, double d, hipStream_t st);
hipError_t launch_gather(double* dst, const int* n, const double* src, const DensBox& b, hipStream_t st);
hipError_t launch_restrict_mean(double* parent, const DensBox& b, const int* m, const double* child, const int* cd,
                                const int* co, hipStream_t st);
hipError_t launch_zero_box(double* out, const double* in, const int* n, const int* lo, const int* m, hipStream_t st);
hipError_t launch_conv_prep(double* a, double* b, double* c, const double* mu, const int* n, const double* par,
                            const DensBox& pb, const int* next_lo, const int* next_m, hipStream_t st);
hipError_t launch_interp_cons(double* out, const int* n, const double* U, const DensBox& b, hipStream_t st);
hipError_t launch_patch_add(double* out, const double* d, const double* C, const int* n, hipStream_t st);
hipError_t launch_restrict_add(double* parent, const DensBox& b, const double* bnd, const int* n, hipStream_t st);
// error reporting shared by the host translation units (sets mg_last_error's message)
int report_error(int code, const char* msg);

}  // namespace mgic
