// Launchers of the bandwidth-bound kernels of the ppwin library.
#pragma once

#include "common.h"

namespace ppw {

// out[p0][p1][p2] = in[d0][d1][d2] with (p0, p1, p2) a permutation of the input axes:
// perm[k] = input axis that becomes output axis k.
void permute3(const double* in, double* out, int d0, int d1, int d2, const int perm[3], hipStream_t s);

// Amplitude strip for occupied rows k0 .. k0+ib-1.  S[(k,x)][(l,y)] = (kx|ly) (rows
// k-local).  Writes (each output optional):
//   tau[(k,x)][(l,y)] = (2 S[(k,x)][(l,y)] - S[(k,y)][(l,x)]) / D,  D = e_k + e_l - e_x - e_y
//   t   = S / D
//   tEv = t * (e_k + e_l - e_y)
//   tEo = t * (e_k - e_x - e_y)
// and per-block partial sums of tau * S into partial[] (one per block, see tau_blocks()).
void tau_strip(const double* S, int o, int v, int k0, int ib, const double* eps_o, const double* eps_v,
               double* tau, double* t, double* tEv, double* tEo, double* partial, hipStream_t s);
long tau_blocks(int o, int v, int ib);
// Same strip built in FP32 (for the reduced-precision product path): tau only, rows of
// ld >= o v values (columns o v .. ld - 1 are not written).
void tau_strip_f32(const float* S, int o, int v, int k0, int ib, const double* eps_o, const double* eps_v,
                   float* tau, long ld, hipStream_t s);

// Deterministic sum of n doubles (single block).
void sum_reduce(const double* x, long n, double* out, hipStream_t s);

// Jacobi/preconditioner diagonals.
//   coul[ia] = (ia|ia) = sum_P B_P,ia^2;  exch[ia] = (ii|aa) = sum_P Boo_P,ii Bvv_P,aa
void diag_integrals(const double* Bov, const double* Boo, const double* Bvv, int o, int v, int naux,
                    double* coul, double* exch, hipStream_t s);
// dA = Delta + c1*(2 coul - exch) [+ A2 diagonal], dB = c1*coul, dS = 1 [- Go_ii - Gv_aa]
void diag_assemble(int o, int v, int order, const double* eps_o, const double* eps_v, const double* coul,
                   const double* exch, const double* Gv, const double* Ev, const double* Go, const double* Eo,
                   double* dA, double* dB, double* dS, hipStream_t s);

// Final combination of one product pass over k particle-hole vectors V ([k][o][v]):
//   AV = Delta*V + 2J + AV_in + [order 2: -P2 + e_i P1 - e_a P3 - P4]
//   BV = 2J + BV_in
//   SV = V - P3 - P1 (order 2), V otherwise
// AV_in/BV_in hold the exchange-type and amplitude terms accumulated by GEMMs.
void sigma_assemble(int o, int v, int k, int order, const double* eps_o, const double* eps_v, const double* V,
                    const double* J, const double* P1, const double* P2, const double* P3, const double* P4,
                    double* AV, double* BV, double* SV, hipStream_t s);

// R[j][s][P][a] (s = 0: Bov + Lambda, s = 1: Bov) for the ring terms of order 2,
// or R[j][P][a] = Bov[P][j][a] when Lam is null.
void build_ring_operand(const double* Bov, const double* Lam, int o, int v, int naux, double* R, hipStream_t s);

// y = alpha*x + beta*y (n elements), and conversions.
void axpby(long n, double alpha, const double* x, double beta, double* y, hipStream_t s);
void to_f32(long n, const double* x, float* y, hipStream_t s);
// y[0..n) = 0 (a kernel, so that it can sit in a captured graph).
void fill_zero(long n, double* y, hipStream_t s);
// y[r][c] = x[r][c] (c < cols) and 0 (cols <= c < ldy) as FP32, for rows r < rows.
void to_f32_rows(long rows, long cols, const double* x, long ldx, float* y, long ldy, hipStream_t s);
// y[c][r] = x[r][c] (r < rows) and 0 (rows <= r < ldy) as FP32, for columns c < cols:
// the transpose of a rows x cols FP64 array into zero-padded FP32 rows.
void transpose_to_f32(long rows, long cols, const double* x, float* y, long ldy, hipStream_t s);
// Excitonic density of states: out[2b] = #pairs with eps_a - eps_i in [edges[b], edges[b+1]),
// out[2b+1] = their sum of squared dipoles (dip nullable).  Device pointers.
void exciton_dos(int o, int v, const double* eo, const double* ev, const double* dip, const double* edges,
                 int n_bins, double* out, hipStream_t s);

void to_f64(long n, const float* x, double* y, hipStream_t s);

// Over a frequency grid omega[n_omega], from n roots (energies e_k > 0, strengths f_k):
//   re + i im = sum_k f_k / (2 e_k) [1 / (w - e_k) - 1 / (w + e_k)],  w = omega + i eta
// (each output nullable), and lor = sum_k f_k (eta / pi) / ((omega - e_k)^2 + eta^2).
// Device pointers; one thread per grid point, roots summed in index order.
void response_on_grid(int n, const double* e, const double* f, int n_omega, const double* omega, double eta,
                      double* re, double* im, double* lor, hipStream_t s);

// Column statistics of k column-vectors of length n stored [k][n] (row-major per vector):
// out[c] = sum_r x[c][r] * y[c][r] (wavefront-level reductions, deterministic order).
void column_dots(const double* x, const double* y, long n, int k, double* out, hipStream_t s);

}  // namespace ppw

namespace ppw {
// out[q][0] = AV[q] + BV[m+q], out[q][1] = BV[q] + AV[m+q]   (M [X;Y] from A, B on X and Y)
// metric: out[q][0] = SV[q], out[q][1] = -SV[m+q]
void combine_pairs(long N, int m, const double* AV, const double* BV, const double* SV, bool metric, double* out,
                   hipStream_t s);
}  // namespace ppw
