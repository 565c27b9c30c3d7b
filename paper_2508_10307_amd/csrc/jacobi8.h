// Parallel cyclic Jacobi for 8x8 Hermitian matrices held in LDS (the basis
// eigenproblems of Eq. 11-12), shared by the basis kernels.
#pragma once
#include "hts_device.h"

namespace hts {

// Partner of index k in round r of the round-robin schedule of the 28 pairs
// of 8 indices (7 rounds of 4 disjoint pairs): 0 stays, 1..7 rotate.
__host__ __device__ constexpr int rr_partner(int k, int r) {
  const int pos = k == 0 ? 0 : 1 + (k - 1 - r + 7) % 7;
  const int pp = 7 - pos;
  return pp == 0 ? 0 : 1 + (pp - 1 + r) % 7;
}

// Parallel cyclic Jacobi on the 8x8 Hermitian covariance matrices (re/im
// parts) held in LDS; on return the diagonal of (mr, mi) holds the
// eigenvalues and (vr, vi) the eigenvectors (columns).  Called by
// every thread of the work group (it synchronises the group): thread 8m + r
// (m < nm) owns row r and column r of matrix m.  Each round rotates the 4
// disjoint pairs (p, q) of the round-robin schedule at once, A <- J^H A J and
// V <- V J, J the product of the 4 rotations
// G = [[c, s], [-s e^{-i phi}, c e^{-i phi}]] on (p, q) that zero
// A(p,q) = |A(p,q)| e^{i phi}.  Both threads of a pair derive the same
// parameters from A; the row update J^H A is written back before the column
// update reads it.  Sweeps end once no pair in any matrix needed a rotation.
__device__ inline void jacobi_herm8_group(double (*mr)[8][8], double (*mi)[8][8], double (*vr)[8][8],
                                   double (*vi)[8][8], int nm) {
  const int t = threadIdx.x;
  const int m = t >> 3, r = t & 7;
  const bool act = m < nm;
  double fn = 0.0;
  if (act) {
    for (int k = 0; k < 8; ++k) {
      vr[m][r][k] = k == r ? 1.0 : 0.0;
      vi[m][r][k] = 0.0;
      fn += mr[m][r][k] * mr[m][r][k] + mi[m][r][k] * mi[m][r][k];
    }
  }
  // Frobenius norm of the matrix: the 8 threads of a matrix are adjacent lanes
#pragma unroll
  for (int o = 1; o < 8; o <<= 1) fn += __shfl_xor(fn, o, 8);
  const double tiny = 1e-17 * sqrt(fn);
  for (int sweep = 0; sweep < 30; ++sweep) {
    int rotated = 0;
    for (int rd = 0; rd < 7; ++rd) {
      const int q = rr_partner(r, rd);
      const int lo = min(r, q), hi = max(r, q);
      double c = 1.0, sn = 0.0, er = 1.0, ei = 0.0;
      double nr[8], ni[8];
      if (act) {
        const double br = mr[m][lo][hi], bi = mi[m][lo][hi];
        const double mag = sqrt(br * br + bi * bi);
        if (!(mag <= tiny)) {   // a NaN rotates too, so it reaches every entry
          rotated = 1;
          const double zeta = (mr[m][hi][hi] - mr[m][lo][lo]) / (2.0 * mag);
          const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          c = 1.0 / sqrt(1.0 + tt * tt);
          sn = tt * c;
          er = br / mag;
          ei = bi / mag;
        }
        // rows lo (x) and hi (y) of G^H A; this thread forms its own row
        const double gqp_r = -sn * er, gqp_i = sn * ei;   // G(q,p) = -s e^{-i phi}
        const double gqq_r = c * er, gqq_i = -c * ei;     // G(q,q) =  c e^{-i phi}
        const double ax = r == lo ? c : sn;               // G(p,p) or G(p,q), real
        const double gr = r == lo ? gqp_r : gqq_r, gi = r == lo ? gqp_i : gqq_i;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const double xr = mr[m][lo][k], xi = mi[m][lo][k];
          const double yr = mr[m][hi][k], yi = mi[m][hi][k];
          nr[k] = ax * xr + gr * yr + gi * yi;
          ni[k] = ax * xi + gr * yi - gi * yr;
        }
      }
      __syncthreads();
      if (act) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          mr[m][r][k] = nr[k];
          mi[m][r][k] = ni[k];
        }
      }
      __syncthreads();
      double wr[8], wi[8];
      if (act) {
        // columns lo (x) and hi (y) of (G^H A) G and of V G; this thread
        // forms its own column
        const double gqp_r = -sn * er, gqp_i = sn * ei;
        const double gqq_r = c * er, gqq_i = -c * ei;
        const double ax = r == lo ? c : sn;
        const double gr = r == lo ? gqp_r : gqq_r, gi = r == lo ? gqp_i : gqq_i;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const double xr = mr[m][k][lo], xi = mi[m][k][lo];
          const double yr = mr[m][k][hi], yi = mi[m][k][hi];
          nr[k] = ax * xr + gr * yr - gi * yi;
          ni[k] = ax * xi + gr * yi + gi * yr;
          const double ur = vr[m][k][lo], ui = vi[m][k][lo];
          const double zr = vr[m][k][hi], zi = vi[m][k][hi];
          wr[k] = ax * ur + gr * zr - gi * zi;
          wi[k] = ax * ui + gr * zi + gi * zr;
        }
      }
      __syncthreads();
      if (act) {
        // exact zeros where the rotation aimed, real diagonal
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          mr[m][k][r] = k == q ? 0.0 : nr[k];
          mi[m][k][r] = k == q || k == r ? 0.0 : ni[k];
          vr[m][k][r] = wr[k];
          vi[m][k][r] = wi[k];
        }
      }
      __syncthreads();
    }
    if (!__syncthreads_or(rotated)) break;
  }
}

}  // namespace hts
