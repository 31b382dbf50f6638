// Restricted additive Schwarz with block ILU(l) subdomain solves (PCSetUp / PCApply).
//
// Paper §3: B^{-1} = sum_i (R_i^0)^T (J_i^delta)^{-1} R_i^delta (eq. (16), transposes in the
// standard place), J_i^delta = R_i^delta J (R_i^delta)^T (eq. (15)), subdomain solve by an
// incomplete LU factorization (§4.3), subdomain matrices in RCM order (§4.5).
//
// Layout: the local rows of all subdomains are concatenated; each subdomain's blocks are
// stored row by row (7x7 row-major FP64).  After factorization a row holds its strict-L
// blocks (unit diagonal implied), the inverse of its U diagonal block, then its strict-U
// blocks.
//
// Schedule: subdomains are independent, so one workgroup owns one subdomain for a whole
// factorization or sweep and walks that subdomain's dependency levels with workgroup
// barriers only -- no grid-wide synchronization and one launch per phase.
//   factor: one wavefront per row, lane (r,c) < 49 owns entry (r,c) of every block of the
//           row; the 7x7 products take a block row from lane registers by shuffles;
//           the pivot block is inverted by Gauss-Jordan with partial pivoting across lanes.
//   sweeps: one wavefront per row, eight block slots per component; the forward sweep
//           gathers R_i^delta v on the fly, the backward sweep applies D_i through shuffles
//           and writes owned rows straight into z (restricted prolongation).
#include "fsi_internal.hpp"

namespace fsi {

static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

__global__ void __launch_bounds__(256) k_ilu_gather(int64_t nb, const int32_t* __restrict__ lsrc,
                                                    const double* __restrict__ vals, double* __restrict__ fac) {
  int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= nb * 49) return;
  const int64_t p = gid / 49;
  const int e = (int)(gid % 49);
  const int src = lsrc[p];
  fac[gid] = src >= 0 ? vals[49 * (size_t)src + e] : 0.0;
}

__global__ void __launch_bounds__(1024) k_ilu_factor(const int32_t* __restrict__ sub_lvl,
                                                     const int32_t* __restrict__ lvl_ptr,
                                                     const int32_t* __restrict__ rows,
                                                     const int32_t* __restrict__ kent_ptr,
                                                     const int32_t* __restrict__ kent_ik,
                                                     const int32_t* __restrict__ kent_dk,
                                                     const int32_t* __restrict__ kent_tptr,
                                                     const int32_t* __restrict__ tri_kj,
                                                     const int32_t* __restrict__ tri_ij,
                                                     const int32_t* __restrict__ ldiag, double* __restrict__ fac,
                                                     double* __restrict__ udiag, int32_t* __restrict__ flags) {
  const int s = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  const int ent = lane < 49 ? lane : 48;  // lanes 49..63 shadow entry 48 and never store
  const bool owner = lane < 49;
  const int rr = ent / 7, cc = ent % 7;
  for (int L = sub_lvl[s]; L < sub_lvl[s + 1]; ++L) {
    const int r1 = lvl_ptr[L + 1];
    for (int q = lvl_ptr[L] + wave; q < r1; q += nwaves) {
      const int i = rows[q];
      for (int ke = kent_ptr[i]; ke < kent_ptr[i + 1]; ++ke) {
        const size_t pik = (size_t)kent_ik[ke] * 49, pdk = (size_t)kent_dk[ke] * 49;
        const double a = fac[pik + ent];
        double arow[7];
#pragma unroll
        for (int m = 0; m < 7; ++m) arow[m] = __shfl(a, rr * 7 + m, 64);
        double l = 0.0;
#pragma unroll
        for (int m = 0; m < 7; ++m) l += arow[m] * fac[pdk + 7 * m + cc];   // L_ik = A_ik D_k
        if (owner) fac[pik + ent] = l;
        double lrow[7];
#pragma unroll
        for (int m = 0; m < 7; ++m) lrow[m] = __shfl(l, rr * 7 + m, 64);
        // A_ij -= L_ik U_kj for the (U_kj, A_ij) pairs of this pivot, four pairs in
        // flight at a time (the U_kj rows are final; the A_ij blocks are distinct)
        int t = kent_tptr[ke];
        const int te = kent_tptr[ke + 1];
        for (; t + 4 <= te; t += 4) {
          size_t pkj[4], pij[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            pkj[u] = (size_t)tri_kj[t + u] * 49;
            pij[u] = (size_t)tri_ij[t + u] * 49;
          }
          double bk[4][7], cur[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
#pragma unroll
            for (int m = 0; m < 7; ++m) bk[u][m] = fac[pkj[u] + 7 * m + cc];
            cur[u] = fac[pij[u] + ent];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            double upd = 0.0;
#pragma unroll
            for (int m = 0; m < 7; ++m) upd += lrow[m] * bk[u][m];
            if (owner) fac[pij[u] + ent] = cur[u] - upd;
          }
        }
        for (; t < te; ++t) {
          const size_t pkj = (size_t)tri_kj[t] * 49, pij = (size_t)tri_ij[t] * 49;
          double u = 0.0;
#pragma unroll
          for (int m = 0; m < 7; ++m) u += lrow[m] * fac[pkj + 7 * m + cc];  // A_ij -= L_ik U_kj
          if (owner) fac[pij + ent] -= u;
        }
      }
      // D_i = A_ii^{-1}: Gauss-Jordan with partial pivoting (first maximum wins)
      const size_t pii = (size_t)ldiag[i] * 49;
      double M = fac[pii + ent];
      if (owner) udiag[49 * (size_t)i + ent] = M;
      double Iv = (rr == cc) ? 1.0 : 0.0;
      bool bad = false;
      for (int p = 0; p < 7; ++p) {
        double colv[7];
#pragma unroll
        for (int m = 0; m < 7; ++m) colv[m] = __shfl(M, m * 7 + p, 64);
        int piv = p;
        double best = fabs(colv[p]);
        for (int m = p + 1; m < 7; ++m)
          if (fabs(colv[m]) > best) { best = fabs(colv[m]); piv = m; }
        if (!(best > 0.0) || !isfinite(best)) bad = true;
        const int srow = (rr == p) ? piv : (rr == piv ? p : rr);
        M = __shfl(M, srow * 7 + cc, 64);
        Iv = __shfl(Iv, srow * 7 + cc, 64);
        const double pv = __shfl(M, p * 7 + p, 64);
        if (rr == p) { M = M / pv; Iv = Iv / pv; }
        const double fct = __shfl(M, rr * 7 + p, 64);
        const double Mp = __shfl(M, p * 7 + cc, 64), Ip = __shfl(Iv, p * 7 + cc, 64);
        if (rr != p) { M = M - fct * Mp; Iv = Iv - fct * Ip; }
      }
      if (bad && lane == 0) atomicOr(&flags[1], 1);
      if (owner) fac[pii + ent] = Iv;
    }
    __syncthreads();
  }
}

// Sweeps: one wavefront per row.  Lane = 8*r + slot: component r (0..6, r = 7 idle) of
// the row, block slot 0..7; slot t accumulates blocks t, t+8, t+16, ... of the row so
// up to eight blocks are in flight per component, then an xor-shuffle tree sums the
// slots.
__global__ void __launch_bounds__(512) k_ilu_fwd(const int32_t* __restrict__ sub_lvl, const int32_t* __restrict__ lvl_ptr,
                                                 const int32_t* __restrict__ rows, const int32_t* __restrict__ lrowptr,
                                                 const int32_t* __restrict__ ldiag, const int32_t* __restrict__ lcol,
                                                 const int32_t* __restrict__ lglob, const double* __restrict__ fac,
                                                 const double* __restrict__ v, double* __restrict__ yl) {
  const int s = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int r = lane >> 3, sl = lane & 7, rr = r < 7 ? r : 6;
  for (int L = sub_lvl[s]; L < sub_lvl[s + 1]; ++L) {
    const int q1 = lvl_ptr[L + 1];
    for (int q = lvl_ptr[L] + wave; q < q1; q += nw) {
      const int i = rows[q];
      const int pd = ldiag[i];
      double acc = 0.0;
#pragma unroll 2
      for (int p = lrowptr[i] + sl; p < pd; p += 8) {
        const double* Lb = fac + 49 * (size_t)p + 7 * rr;
        const double* yk = yl + 7 * (size_t)lcol[p];
#pragma unroll
        for (int m = 0; m < 7; ++m) acc += Lb[m] * yk[m];
      }
      acc += __shfl_xor(acc, 1, 64);
      acc += __shfl_xor(acc, 2, 64);
      acc += __shfl_xor(acc, 4, 64);
      if (sl == 0 && r < 7) yl[7 * (size_t)i + r] = v[7 * (size_t)lglob[i] + r] - acc;
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(512) k_ilu_bwd(const int32_t* __restrict__ sub_lvl, const int32_t* __restrict__ lvl_ptr,
                                                 const int32_t* __restrict__ rows, const int32_t* __restrict__ lrowptr,
                                                 const int32_t* __restrict__ ldiag, const int32_t* __restrict__ lcol,
                                                 const int32_t* __restrict__ lglob, const uint8_t* __restrict__ lowned,
                                                 const double* __restrict__ fac, double* __restrict__ yl,
                                                 double* __restrict__ z) {
  const int s = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int r = lane >> 3, sl = lane & 7, rr = r < 7 ? r : 6;
  for (int L = sub_lvl[s]; L < sub_lvl[s + 1]; ++L) {
    const int q1 = lvl_ptr[L + 1];
    for (int q = lvl_ptr[L] + wave; q < q1; q += nw) {
      const int i = rows[q];
      const int pd = ldiag[i];
      double acc = 0.0;
#pragma unroll 2
      for (int p = pd + 1 + sl; p < lrowptr[i + 1]; p += 8) {
        const double* Ub = fac + 49 * (size_t)p + 7 * rr;
        const double* xj = yl + 7 * (size_t)lcol[p];
#pragma unroll
        for (int m = 0; m < 7; ++m) acc += Ub[m] * xj[m];
      }
      acc += __shfl_xor(acc, 1, 64);
      acc += __shfl_xor(acc, 2, 64);
      acc += __shfl_xor(acc, 4, 64);
      const double t = yl[7 * (size_t)i + rr] - acc;   // component rr of y_i - sum U_ij x_j
      const double* D = fac + 49 * (size_t)pd + 7 * rr;
      double x = 0.0;
#pragma unroll
      for (int c = 0; c < 7; ++c) x += D[c] * __shfl(t, 8 * c, 64);
      if (sl == 0 && r < 7) {
        yl[7 * (size_t)i + r] = x;
        if (lowned[i]) z[7 * (size_t)lglob[i] + r] = x;
      }
    }
    __syncthreads();
  }
}

hipError_t launch_pc_setup(fsi_solver* s) {
  if (s->NB == 0) return hipSuccess;
  hipLaunchKernelGGL(k_ilu_gather, dim3(nblk(s->NB * 49, 256)), dim3(256), 0, s->stream, s->NB, s->lsrc, s->vals,
                     s->fac);
  FSI_PROF_LAUNCH(s, "ilu_factor",
                  hipLaunchKernelGGL(k_ilu_factor, dim3(s->h.ns), dim3(1024), 0, s->stream, s->fwd_sub_lvl,
                                     s->fwd_lvl_ptr, s->fwd_rows, s->kent_ptr, s->kent_ik, s->kent_dk, s->kent_tptr,
                                     s->tri_kj, s->tri_ij, s->ldiag, s->fac, s->udiag, s->flags));
  return hipGetLastError();
}

hipError_t launch_pc_apply(fsi_solver* s, const double* v, double* z) {
  FSI_PROF_LAUNCH(s, "ilu_fwd",
                  hipLaunchKernelGGL(k_ilu_fwd, dim3(s->h.ns), dim3(512), 0, s->stream, s->fwd_sub_lvl, s->fwd_lvl_ptr,
                                     s->fwd_rows, s->lrowptr, s->ldiag, s->lcol, s->lglob, s->fac, v, s->ylocal));
  FSI_PROF_LAUNCH(s, "ilu_bwd",
                  hipLaunchKernelGGL(k_ilu_bwd, dim3(s->h.ns), dim3(512), 0, s->stream, s->bwd_sub_lvl, s->bwd_lvl_ptr,
                                     s->bwd_rows, s->lrowptr, s->ldiag, s->lcol, s->lglob, s->lowned, s->fac,
                                     s->ylocal, z));
  return hipGetLastError();
}

}  // namespace fsi
