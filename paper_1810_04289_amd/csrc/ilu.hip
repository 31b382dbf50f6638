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
//   sweeps: one wavefront per row, lane (r,c) < 56 owns entry (r,c) of each block of the
//           row (coalesced block loads); results of earlier levels come from LDS slots; the
//           forward sweep gathers R_i^delta v on the fly, the backward sweep applies D_i and
//           writes owned rows straight into z (restricted prolongation).
#include <algorithm>
#include <type_traits>

#include "fsi_internal.hpp"

namespace fsi {

static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }
// A dispatch packet holds the grid size as a 32-bit count of work-items, so launches over
// per-entry ranges (49 per block, past 2^32 at the largest subdomain sets) stride over a
// capped grid instead of launching one work-item per entry.
static inline unsigned nblk_stride(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return (unsigned)(b < (int64_t(1) << 20) ? (b > 0 ? b : 1) : (int64_t(1) << 20));
}

template <typename T>
__global__ void __launch_bounds__(256) k_ilu_gather(int64_t nb, const int32_t* __restrict__ lsrc,
                                                    const double* __restrict__ vals, T* __restrict__ fac) {
  const int64_t n = nb * 49, stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; gid < n; gid += stride) {
    const int64_t p = gid / 49;
    const int e = (int)(gid - 49 * p);
    const int src = lsrc[p];
    fac[gid] = src >= 0 ? (T)vals[49 * (size_t)src + e] : (T)0;
  }
}

// Wavefront-scope ordering of LDS accesses between lanes of one wavefront (LDS operations
// of a wavefront are processed in order; the fences keep the compiler from reordering).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Raw buffer loads: a resource spans exactly the bytes a task may read, and the hardware
// returns 0 for a lane whose offset (vector offset + immediate) falls outside it, without
// touching memory.  Padding lanes use an offset that is always outside.
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
constexpr int kBufFlags = 0x00020000;  // raw 32-bit data format (gfx9 family)
constexpr int kOutside = (int)0x80000000u;

// The arguments are uniform; readfirstlane keeps the descriptor in scalar registers even
// where the compiler computed a piece of it with vector instructions.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t span_rsrc(const void* p, int bytes) {
  const uint64_t a = (uint64_t)p;
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)a);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(a >> 32));
  void* q = (void*)(((uint64_t)hi << 32) | lo);
  return __builtin_amdgcn_make_buffer_rsrc(q, (short)0, __builtin_amdgcn_readfirstlane(bytes), kBufFlags);
}

__device__ __forceinline__ double span_load_f64(__amdgpu_buffer_rsrc_t r, int voff) {
  const u32x2_t v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, 0, 0);
  return __hiloint2double((int)v.y, (int)v.x);
}

__device__ __forceinline__ void span_store_f64(__amdgpu_buffer_rsrc_t r, int voff, double x) {
  u32x2_t v;
  v.x = (unsigned)__double2loint(x);
  v.y = (unsigned)__double2hiint(x);
  __builtin_amdgcn_raw_buffer_store_b64(v, r, voff, 0, 0);
}

// The factorization's arithmetic type: FP64, or FP32 for factors computed in FP32.
template <typename T>
__device__ __forceinline__ T span_load_t(__amdgpu_buffer_rsrc_t r, int voff);
template <>
__device__ __forceinline__ double span_load_t<double>(__amdgpu_buffer_rsrc_t r, int voff) {
  return span_load_f64(r, voff);
}
template <>
__device__ __forceinline__ float span_load_t<float>(__amdgpu_buffer_rsrc_t r, int voff) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, 0, 0));
}
__device__ __forceinline__ void span_store_t(__amdgpu_buffer_rsrc_t r, int voff, double x) { span_store_f64(r, voff, x); }
__device__ __forceinline__ void span_store_t(__amdgpu_buffer_rsrc_t r, int voff, float x) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(x), r, voff, 0, 0);
}
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

constexpr int kFacDepth = 3;  // factorization groups in flight per wavefront
constexpr int kWaitVmcnt0 = 0x0F70;  // s_waitcnt operand: vmcnt(0), other counters free

struct FacDesc {  // one factorization group, uniform across the wavefront (see fsi_internal.hpp)
  int ublock, dk, moff, flags;
};

__device__ __forceinline__ FacDesc desc_get(const int4& c, int l) {
  return FacDesc{__builtin_amdgcn_readlane(c.x, l), __builtin_amdgcn_readlane(c.y, l),
                 __builtin_amdgcn_readlane(c.z, l), __builtin_amdgcn_readlane(c.w, l)};
}

constexpr int kFacCodeLead = 2;  // groups between a group's code loads and its block loads

template <typename T>
struct FacGroup {     // what a group reads from memory
  T u[2][7];          // lane q < 63: U_kj[m][q % 7] of the group's blocks q / 7 and 9 + q / 7
  T d;                // lane e < 49: entry e of D_k
  int pos[2];         // 1 + position of A_ij of those blocks in row i, or 0 (no block)
};

// A group's codes: for lane q, those of its blocks q / 7 and 9 + q / 7, each (t << 16) | pos
// with t the block's index in U_k and pos its position in row i plus one, or 0 past the
// group's blocks (the resource ends with them, so those lanes read 0 without touching memory).
__device__ __forceinline__ void fac_codes_load(int (&c)[2], const FacDesc& F, bool real,
                                               const int32_t* __restrict__ codes, int lane) {
  const int nblk = real ? (F.flags >> 1) & 31 : 0;
  const __amdgpu_buffer_rsrc_t rm = span_rsrc(codes + F.moff, 4 * nblk);
#pragma unroll
  for (int h = 0; h < 2; ++h)
    c[h] = (int)__builtin_amdgcn_raw_buffer_load_b32(rm, 4 * (lane / 7) + 4 * kFacHalf * h, 0, 0);
}

// Its blocks of U_k (at the codes' indices) and D_k.  The blocks' resource runs from U_k's
// first block to at most 65535 blocks on, and never past the end of the factors.
template <typename T>
__device__ __forceinline__ void fac_blocks_load(FacGroup<T>& G, const int (&c)[2], const FacDesc& F, bool real,
                                                const T* __restrict__ fac, int64_t nbk, bool qlane, int qc,
                                                int voff_d) {
  constexpr int W = (int)sizeof(T);
  const int64_t room = real ? nbk - F.ublock : 0;
  const __amdgpu_buffer_rsrc_t ru =
      span_rsrc(fac + 49 * (size_t)F.ublock, 49 * W * (int)(room < 65535 ? room : 65535));
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int voff = (qlane && c[h] != 0) ? W * (49 * (c[h] >> 16) + qc) : kOutside;
#pragma unroll
    for (int m = 0; m < 7; ++m) G.u[h][m] = span_load_t<T>(ru, voff + 7 * W * m);
    G.pos[h] = c[h] & 0xffff;
  }
  G.d = span_load_t<T>(span_rsrc(fac + 49 * (size_t)F.dk, real ? 49 * W : 0), voff_d);
}

// Factorization of one subdomain per workgroup, block IKJ order, one row at a time per
// wavefront.  The row being factored is staged in the wavefront's LDS slice of `slice`
// blocks; the blocks of a longer row past the slice stay in global memory and are updated
// there (read-modify-write by the row's own wavefront, its stores completed before it
// reads them again), so that a slice need not fit the longest row.
// Its work is a list of groups built on the host: for each pivot k (ascending), the blocks
// U_kj whose A_ij is in row i's pattern, in groups of up to 18 (one group if there are
// none); the others would update nothing.  The first group of a pivot forms
// L_ik = A_ik D_k with lane e < 49 holding entry e, writes it back and reads it into every
// lane; each group then applies A_ij -= L_ik U_kj to its blocks, lane q < 63 holding column
// q % 7 of blocks q / 7 and 9 + q / 7 (98 FMAs and 14 LDS read-modify-writes per lane; a
// group of at most 9 blocks skips the second half).  A group's codes (which blocks, and
// where in row i) are loaded kFacCodeLead groups before its blocks, and its blocks while
// group t - P + 1 computes, into P rotating register sets; the group descriptors arrive
// 64 at a time, one per lane, broadcast by readlane.
//
// Schedule.  The rows go to the wavefronts round-robin in level order, and each wavefront
// works through its rows as far ahead as their pivots allow: a group may start once its
// pivot row is final.  There are no level barriers.  Each wavefront publishes in LDS a
// progress level p_w such that all of its rows below level p_w are final (the level of its
// next unfinished row), raised after a row's write-back has completed; a group whose pivot
// row has level l waits until min_w p_w > l.  Rows depend only on rows of lower levels, and
// the wavefront with the smallest p_w is working on a row whose pivots are all below that
// level, so it always proceeds: the waits cannot form a cycle.  Each wait is bounded all
// the same; a wavefront that exceeds the bound raises an error flag and stops waiting, so
// that the kernel still ends (with its factors marked invalid).
template <int NT, int P, typename T>
__global__ void __launch_bounds__(NT) k_ilu_factor(const int32_t* __restrict__ nphase,
                                                   const int32_t* __restrict__ fw_ptr,
                                                   const int32_t* __restrict__ fw_row,
                                                   const int32_t* __restrict__ fw_lvl,
                                                   const int32_t* __restrict__ lrowptr,
                                                   const int32_t* __restrict__ fgrp_ptr,
                                                   const int4* __restrict__ fgrp,
                                                   const int32_t* __restrict__ fgrp_lvl,
                                                   const int32_t* __restrict__ umap,
                                                   const int64_t* __restrict__ umap_row, int64_t nbk,
                                                   const int32_t* __restrict__ ldiag, T* __restrict__ fac,
                                                   T* __restrict__ udiag, int32_t* __restrict__ flags,
                                                   int slice, int wait_limit) {
  // Every entry of a block product is a sum over m in ascending order from 0, each term
  // added with one rounding (fused multiply-add), and nothing else is fused or reordered.
  // The block elimination of the wall rows amplifies a difference of one rounding in its
  // input to about 1e-4 in its factors, so only the same rounded operations give factors
  // that are reproducible anywhere else.
#pragma clang fp contract(off)
  extern __shared__ double lds_d[];
  T* lds = reinterpret_cast<T*>(lds_d);
  constexpr int W = (int)sizeof(T);
  constexpr int NW = NT / 64;
  const int s = blockIdx.x;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int ent = lane < 49 ? lane : 48;  // lanes 49..63 shadow entry 48 and never store
  const bool owner = lane < 49;
  const int rr = ent / 7, cc = ent % 7;
  const int qc = lane % 7;  // group lanes: column (of blocks lane / 7 and 9 + lane / 7)
  const bool qlane = lane < 7 * kFacHalf;
  const int voff_d = owner ? W * ent : kOutside;
  T* row = lds + (size_t)wave * (slice * 49 + 56);
  T* dsc = row + (size_t)slice * 49;  // D_k of the current pivot, then L_ik
  const int nL = nphase[s];
  const int wb = fw_ptr[s * NW + wave], we = fw_ptr[s * NW + wave + 1];
  __shared__ int prog[NW];  // progress levels of the wavefronts
  if (lane == 0) prog[wave] = wb < we ? fw_lvl[wb] : nL;
  __syncthreads();
  int seen = 0;      // a lower bound of min_w p_w (the levels only grow)
  bool live = true;  // false once a wait has exceeded its bound
  // wait until every row of level <= l is final; the acquire fence keeps the pivot row's
  // loads after the wait
  auto wait_final = [&](int l) {
    if (l < seen || !live) return;
    for (int spins = 0;; ++spins) {
      int m = nL;
#pragma unroll
      for (int w = 0; w < NW; ++w) m = min(m, __hip_atomic_load(&prog[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
      seen = __builtin_amdgcn_readfirstlane(m);
      if (l < seen) break;
      if (spins == wait_limit) {
        live = false;
        if (lane == 0) atomicOr(&flags[2], 1);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  };
  for (int rw = wb; rw < we; ++rw) {
    // row metadata is uniform across the wavefront: keep it in scalar registers
    const int i = __builtin_amdgcn_readfirstlane(fw_row[rw]);
    const int Li = __builtin_amdgcn_readfirstlane(fw_lvl[rw]);
    const int rb = __builtin_amdgcn_readfirstlane(lrowptr[i]);
    const int nbe = (__builtin_amdgcn_readfirstlane(lrowptr[i + 1]) - rb) * 49;
    const int nbs = nbe < slice * 49 ? nbe : slice * 49;  // entries staged in LDS
    const bool spill = nbe > nbs;                         // blocks past the slice in memory
    const size_t gb = (size_t)rb * 49;
    T* grow = fac + gb;  // the row in memory
    // the row's blocks past the slice are read and written through buffer instructions
    const __amdgpu_buffer_rsrc_t rrow = span_rsrc(grow, W * nbe);
    // this row's part of the U-position map (uniform: kept in scalar registers)
    const int64_t ub = umap_row[i];
    const int32_t* urow = umap + (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)ub)) |
                                           ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(ub >> 32)) << 32));
    const int g0 = __builtin_amdgcn_readfirstlane(fgrp_ptr[i]);
    const int ng = __builtin_amdgcn_readfirstlane(fgrp_ptr[i + 1]) - g0;
    // c0 holds groups [cb, cb + 64) (descriptors, and pivot levels in v0) and c1 / v1 the
    // next chunk; consecutive chunks overlap by P - 1 + Q groups, so group t and the groups
    // t + P - 1 and t + P - 1 + Q loaded with it always share c0
    constexpr int Q = kFacCodeLead;
    static_assert(Q >= 1 && Q <= P - 1, "a code slot is reused P groups later");
    constexpr int kStride = 64 - (P - 1 + Q);
    auto chunk = [&](int t) { return fgrp[ng > 0 ? g0 + (t + lane < ng ? t + lane : ng - 1) : 0]; };
    auto lchunk = [&](int t) { return fgrp_lvl[ng > 0 ? g0 + (t + lane < ng ? t + lane : ng - 1) : 0]; };
    int cb = 0;
    int4 c0 = chunk(0), c1 = chunk(kStride);
    int v0 = lchunk(0), v1 = lchunk(kStride);
    // stage the row: all loads of a round issued before its LDS writes
    for (int e0 = 0; e0 < nbs; e0 += 64 * 8) {
      T tmp[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + lane + 64 * u;
        tmp[u] = grow[e < nbs ? e : nbs - 1];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + lane + 64 * u;
        if (e < nbs) row[e] = tmp[u];
      }
    }
    wave_lds_sync();
    T lrow[7][7];  // L_ik of the current pivot, all entries in every lane
    auto consume = [&](const FacGroup<T>& G, const FacDesc& F) {
      const int pik = F.flags >> 6;
      if (F.flags & 1) {  // first group of the pivot: L_ik = A_ik D_k
        if (owner) dsc[ent] = G.d;
        wave_lds_sync();
        T l = (T)0;
        if (pik < slice) {
#pragma unroll
          for (int m = 0; m < 7; ++m) l = fma_t(row[pik * 49 + 7 * rr + m], dsc[7 * m + cc], l);
        } else {
#pragma unroll
          for (int m = 0; m < 7; ++m)
            l = fma_t(span_load_t<T>(rrow, W * (pik * 49 + 7 * rr + m)), dsc[7 * m + cc], l);
        }
        wave_lds_sync();
        if (owner) {
          dsc[ent] = l;
          if (pik < slice) row[pik * 49 + ent] = l;
          else span_store_t(rrow, W * (pik * 49 + ent), l);
        }
        wave_lds_sync();
#pragma unroll
        for (int r = 0; r < 7; ++r)
#pragma unroll
          for (int m = 0; m < 7; ++m) lrow[r][m] = dsc[7 * r + m];
      }
      // A_ij -= L_ik U_kj, column qc of the two blocks: every row's sum in ascending m; the
      // loops run over m outside so that the fourteen sums interleave instead of waiting on
      // one another.  The two blocks are different blocks
      // of row i, so both are read before either is written.
      auto update = [&](auto nh_c) {
        constexpr int NH = decltype(nh_c)::value;  // halves with blocks
        T acc[NH][7];
#pragma unroll
        for (int h = 0; h < NH; ++h)
#pragma unroll
          for (int r = 0; r < 7; ++r) acc[h][r] = (T)0;
#pragma unroll
        for (int m = 0; m < 7; ++m)
#pragma unroll
          for (int h = 0; h < NH; ++h)
#pragma unroll
            for (int r = 0; r < 7; ++r) acc[h][r] = fma_t(lrow[r][m], G.u[h][m], acc[h][r]);
        T av[NH][7];
#pragma unroll
        for (int h = 0; h < NH; ++h) {
          const int p = G.pos[h] - 1;
          if (qlane && p >= 0 && p < slice) {
#pragma unroll
            for (int r = 0; r < 7; ++r) av[h][r] = row[p * 49 + qc + 7 * r];
          }
        }
#pragma unroll
        for (int h = 0; h < NH; ++h) {
          const int p = G.pos[h] - 1;
          if (qlane && p >= 0 && p < slice) {
#pragma unroll
            for (int r = 0; r < 7; ++r) row[p * 49 + qc + 7 * r] = av[h][r] - acc[h][r];
          } else if (qlane && p >= slice) {
            const int o = W * (p * 49 + qc);
#pragma unroll
            for (int r = 0; r < 7; ++r)
              span_store_t(rrow, o + 7 * W * r, span_load_t<T>(rrow, o + 7 * W * r) - acc[h][r]);
          }
        }
      };
      if (((F.flags >> 1) & 31) > kFacHalf) update(std::integral_constant<int, 2>());
      else update(std::integral_constant<int, 1>());
      // a later group may read back what this one stored past the slice
      if (spill) __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
      wave_lds_sync();
    };
    if (ng > 0) {
      // step t loads the codes of group t + P - 1 + Q, then the blocks of group t + P - 1
      // (codes loaded Q steps before), then computes group t; code set g % P is next
      // written for group g + P, at step g + 1 - Q, after its use at step g - P + 1
      FacGroup<T> buf[P];
      int cod[P][2];
      auto step_loads = [&](int gc, int cslot, int gb, int bslot) {
        const int uc = gc < ng ? gc : ng - 1;
        fac_codes_load(cod[cslot], desc_get(c0, uc - cb), gc < ng, urow, lane);
        if (gb >= 0) {
          const int ubk = gb < ng ? gb : ng - 1;
          wait_final(__builtin_amdgcn_readlane(v0, ubk - cb));  // pivot row final before its blocks are read
          fac_blocks_load(buf[bslot], cod[bslot], desc_get(c0, ubk - cb), gb < ng, fac, nbk, qlane, qc, voff_d);
        }
      };
#pragma unroll
      for (int t = -(P - 1 + Q); t < 0; ++t) step_loads(t + P - 1 + Q, (t + P - 1 + Q) % P, t + P - 1, (t + 2 * P - 1) % P);
      for (int t0 = 0; t0 < ng; t0 += P) {
#pragma unroll
        for (int k = 0; k < P; ++k) {
          const int t = t0 + k;
          if (t < ng && t + P - 1 + Q - cb == 64) {  // the chunk at cb + kStride starts at group t
            c0 = c1;
            v0 = v1;
            cb += kStride;
            c1 = chunk(cb + kStride);
            v1 = lchunk(cb + kStride);
          }
          step_loads(t + P - 1 + Q, (k + P - 1 + Q) % P, t + P - 1, (k + P - 1) % P);
          if (t < ng) consume(buf[k], desc_get(c0, t - cb));
        }
      }
    }
    // D_i = A_ii^{-1}: Gauss-Jordan with partial pivoting (first maximum wins) on the
    // equilibrated block Ah = R A C, R and C powers of two that bring each row's and then
    // each column's largest entry into [1, 2); then A^{-1} = C Ah^{-1} R.  The scalings are
    // exact: the inverse is the same, only its rounding improves (the wall's pivot blocks
    // mix entries from 1e-10 to 1e4).
    const int pdb = __builtin_amdgcn_readfirstlane(ldiag[i]) - rb;  // block position of A_ii
    T M = pdb < slice ? row[pdb * 49 + ent] : span_load_t<T>(rrow, W * (pdb * 49 + ent));
    if (owner) udiag[49 * (size_t)i + ent] = M;
    bool bad = false;
    T rs, cs;  // scale of this lane's row (r_rr) and column (c_cc)
    {
      T mx = (T)0;
#pragma unroll
      for (int m = 0; m < 7; ++m) mx = fmax(mx, fabs(__shfl(M, 7 * rr + m, 64)));
      if (!(mx > 0.0) || !isfinite(mx)) bad = true;
      int e;
      frexp(mx, &e);
      rs = (T)1 / ldexp((T)1, e - 1);
      const T Mr = M * rs;
      mx = (T)0;
#pragma unroll
      for (int m = 0; m < 7; ++m) mx = fmax(mx, fabs(__shfl(Mr, 7 * m + cc, 64)));
      if (!(mx > 0.0)) bad = true;
      frexp(mx, &e);
      cs = (T)1 / ldexp((T)1, e - 1);
      M = Mr * cs;
    }
    T Iv = (rr == cc) ? (T)1 : (T)0;
    for (int p = 0; p < 7; ++p) {
      T colv[7];
#pragma unroll
      for (int m = 0; m < 7; ++m) colv[m] = __shfl(M, m * 7 + p, 64);
      int pr = p;
      T best = fabs(colv[p]);
      for (int m = p + 1; m < 7; ++m)
        if (fabs(colv[m]) > best) { best = fabs(colv[m]); pr = m; }
      if (!(best > 0.0) || !isfinite(best)) bad = true;
      const int srow = (rr == p) ? pr : (rr == pr ? p : rr);
      M = __shfl(M, srow * 7 + cc, 64);
      Iv = __shfl(Iv, srow * 7 + cc, 64);
      const T pv = __shfl(M, p * 7 + p, 64);
      if (rr == p) { M = M / pv; Iv = Iv / pv; }
      const T fct = __shfl(M, rr * 7 + p, 64);
      const T Mp = __shfl(M, p * 7 + cc, 64), Ip = __shfl(Iv, p * 7 + cc, 64);
      if (rr != p) { M = M - fct * Mp; Iv = Iv - fct * Ip; }
    }
    // entry (rr, cc) of A^{-1} is c_rr Ah^{-1}(rr, cc) r_cc: c_rr from lane (0, rr), r_cc
    // from lane (cc, 0)
    Iv = __shfl(cs, rr, 64) * Iv * __shfl(rs, 7 * cc, 64);
    if (bad && lane == 0) {
      atomicOr(&flags[1], 1);
      atomicMax(&flags[4], i + 1);  // i: the concatenated local row
      atomicMax(&flags[5], 0x7fffffff - i);
      atomicAdd(&flags[6], 1);
    }
    wave_lds_sync();
    if (owner) {
      if (pdb < slice) row[pdb * 49 + ent] = Iv;
      else span_store_t(rrow, W * (pdb * 49 + ent), Iv);
    }
    wave_lds_sync();
    // write back the staged part; blocks past the slice are already in place
    for (int e0 = 0; e0 < nbs; e0 += 64 * 8) {
      T tmp[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + lane + 64 * u;
        tmp[u] = row[e < nbs ? e : nbs - 1];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + lane + 64 * u;
        if (e < nbs) grow[e] = tmp[u];
      }
    }
    // release: once the write-back has completed, raise the progress level to the next
    // row's level (unchanged when that row is of the same level)
    const int next_lvl = rw + 1 < we ? __builtin_amdgcn_readfirstlane(fw_lvl[rw + 1]) : nL;
    if (next_lvl > Li) {
      __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      if (lane == 0) __hip_atomic_store(&prog[wave], next_lvl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
  }
}

// LDS of the factorization: per wavefront a slice of `slice` staged blocks plus D_k, and 64 B
// for the progress levels.  As many wavefronts (up to four) as slices for the longest row
// fit; but when four slices of at least 90% of the longest row fit, four wavefronts with
// such slices, the few longer rows keeping their tails in memory.  elem_bytes: 8 for an
// FP64 factorization, 4 for FP32.
FacLayout fac_layout(int max_rowblk, int elem_bytes) {
  const size_t cap = 160 * 1024 - 64;
  auto per_wave = [&](size_t blocks) { return (blocks * 49 + 56) * (size_t)elem_bytes; };
  const int full = (int)std::min<size_t>(4, cap / per_wave((size_t)max_rowblk));
  if (full >= 4) return FacLayout{4, max_rowblk};
  const int s4 = (int)((cap / 4 / (size_t)elem_bytes - 56) / 49);
  if (10 * s4 >= 9 * max_rowblk) return FacLayout{4, s4};
  return FacLayout{full, max_rowblk};
}

template <typename T>
static hipError_t pc_setup_t(fsi_solver* s, T* fac, T* udiag) {
  hipLaunchKernelGGL(k_ilu_gather<T>, dim3(nblk_stride(s->NB * 49)), dim3(256), 0, s->stream, s->NB, s->lsrc,
                     s->vals, fac);
  // up to four row-staging wavefronts per workgroup, as many as the longest row allows (the
  // rows were dealt to that many wavefronts at create)
  const FacLayout fl = fac_layout(s->max_rowblk, (int)sizeof(T));
  const int waves = s->fac_nw;
  if (waves < 1 || waves != fl.waves || fl.slice < 1) return hipErrorInvalidConfiguration;
  const size_t per_wave = ((size_t)fl.slice * 49 + 56) * sizeof(T);
  const size_t lds = per_wave * waves;
  auto go = [&](auto kern, int nt) -> hipError_t {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    FSI_PROF_LAUNCH(s, "ilu_factor",
                    hipLaunchKernelGGL(kern, dim3(s->h.ns), dim3(nt), lds, s->stream, s->fwd_nphase, s->fw_ptr,
                                       s->fw_row, s->fw_lvl, s->lrowptr, s->fgrp_ptr, s->fgrp, s->fgrp_lvl, s->umap,
                                       s->umap_row, s->NB,
                                       s->ldiag, fac, udiag, s->flags, fl.slice, s->wait_limit));
    return hipSuccess;
  };
  constexpr int P = kFacDepth;
  hipError_t e = waves >= 4 ? go(k_ilu_factor<256, P, T>, 256) : waves == 3 ? go(k_ilu_factor<192, P, T>, 192)
                 : waves == 2 ? go(k_ilu_factor<128, P, T>, 128) : go(k_ilu_factor<64, P, T>, 64);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

hipError_t launch_pc_setup(fsi_solver* s) {
  if (s->NB == 0) return hipSuccess;
  if (s->opts.precision == FSI_PREC_FP32_FACTOR) return pc_setup_t<float>(s, s->fac32, s->udiag32);
  return pc_setup_t<double>(s, s->fac, s->udiag);
}

// Sweeps: one wavefront per row.  Lane = 8*r + c holds entry (r, c) of a 7x7 block
// (c = 7 and r = 7 idle), so one load instruction reads a whole 392-byte block
// contiguously; the row's blocks are multiplied by the column rows' values and summed
// over blocks per lane, then a DPP tree sums the eight lanes of each row r.
//
// Level results travel through LDS: each row whose value is read later in the same sweep
// owns an LDS slot from its level to its last reader's level (slots assigned on the host
// by interval colouring; a few hundred slots per subdomain).
//
// Levels (phases) are ordered without barriers.  Each wavefront publishes in LDS the phase
// of its next unfinished row: all of its rows below that phase are finished.  A task of
// phase p waits until every wavefront has published at least p, so the rows it reads have
// been written; a row taking over a slot has a phase above the slot's last reader's, so
// that reader is finished too.  The wavefront with the smallest published phase can always
// run its next task (a task's phase never exceeds its row's), so the waits cannot form a
// cycle; each is bounded all the same, and past the bound the wavefront sets an error flag
// and stops waiting.  Only LDS is ordered, so global loads stay in flight across the waits.
//
// Nothing a wavefront loads from memory depends on values computed in the sweep, so the
// sweep is a pipeline over the wavefront's task list: the task metadata arrive 64 tasks at
// a time (one task per lane, broadcast by readlane) and the block values, the column
// rows' LDS slots and the row's input of task t + D - 1 are requested right after task t
// is computed and its phase released, into D rotating register sets.  Every task issues the same number of loads
// (blocks beyond the task's range read 0), so the compiler's in-order memory counter waits
// only for the set about to be used.  A row longer than MB blocks is split into consecutive
// tasks of at most MB blocks that carry their partial sums in registers; only the last one
// finishes the row (the backward sweep takes the chunk next to D_i last).
// Factor storage of the sweeps: FP64 (computed in FP64), or the FP64 factors rounded to
// FP32 or BF16 with FP32 arithmetic.  Value<S>::C is the arithmetic type.
struct bf16_t {
  uint16_t bits;
};
template <typename S>
struct Value;
template <>
struct Value<double> {
  using C = double;
  __device__ static double load(__amdgpu_buffer_rsrc_t r, int voff) { return span_load_f64(r, voff); }
};
template <>
struct Value<float> {
  using C = float;
  __device__ static float load(__amdgpu_buffer_rsrc_t r, int voff) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, 0, 0));
  }
};
template <>
struct Value<bf16_t> {
  using C = float;
  __device__ static float load(__amdgpu_buffer_rsrc_t r, int voff) {
    return __uint_as_float((uint32_t)__builtin_amdgcn_raw_buffer_load_b16(r, voff, 0, 0) << 16);
  }
};

template <int CTRL>
__device__ __forceinline__ float dpp_mov(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// sum over the eight lanes of an aligned group of eight (xor 1, xor 2, then the mirror
// lane of the other half)
template <typename C>
__device__ __forceinline__ C sum8(C v) {
  v += dpp_mov<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_mov<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_mov<0x141>(v);  // row_half_mirror
  return v;
}

struct TaskMeta {  // one task, uniform across the wavefront
  // phase: when the task may run (the row's own phase for the task that finishes the row,
  // earlier for the leading tasks of a split row); row_phase: the row's own phase
  int row, vtx, first, last, slot, phase, flags, row_phase;
};

struct TaskChunk {  // lane j: task base + j
  int4 m, a;
};

__device__ __forceinline__ TaskChunk load_chunk(const int4* __restrict__ task, const int4* __restrict__ aux, int t,
                                                int te, int lane) {
  const int q = t + lane < te ? t + lane : te - 1;
  return TaskChunk{task[q], aux[q]};
}

__device__ __forceinline__ TaskMeta chunk_get(const TaskChunk& c, int l) {
  return TaskMeta{__builtin_amdgcn_readlane(c.m.x, l), __builtin_amdgcn_readlane(c.m.y, l),
                  __builtin_amdgcn_readlane(c.m.z, l), __builtin_amdgcn_readlane(c.m.w, l),
                  __builtin_amdgcn_readlane(c.a.x, l), __builtin_amdgcn_readlane(c.a.y, l),
                  __builtin_amdgcn_readlane(c.a.z, l), __builtin_amdgcn_readlane(c.a.w, l)};
}

template <typename C, int MB>
struct TaskData {
  C A[MB];   // entry (r, c) of the task's blocks; 0 beyond its range and on padding lanes
  int ls;    // lane b < MB: LDS byte offset of the column row of block b (0 beyond the range)
  C base;    // forward: v of the vertex (component r); backward: y_i (component r)
  C D;       // backward: entry (r, c) of D_i (0 on padding lanes)
};

// voff: sizeof(S) * (7r + c) on the 49 block lanes, kOutside on padding lanes
template <typename S, int BWD, int MB>
__device__ __forceinline__ void task_load(TaskData<typename Value<S>::C, MB>& P, const TaskMeta& T,
                                          const int32_t* __restrict__ lslot, const S* __restrict__ fac,
                                          const double* __restrict__ v, const typename Value<S>::C* yl, int lane,
                                          int voff, int r) {
  using C = typename Value<S>::C;
  constexpr int BB = 49 * (int)sizeof(S);  // bytes per block
  const int first = T.first;
  const int nb = T.last - first;
  // one resource per group of eight blocks keeps every block offset in the immediate field
#pragma unroll
  for (int g = 0; g < MB; g += 8) {
    const __amdgpu_buffer_rsrc_t ra = span_rsrc(fac + 49 * (size_t)(first + g), nb > g ? BB * (nb - g) : 0);
#pragma unroll
    for (int u = 0; u < 8 && g + u < MB; ++u) P.A[g + u] = Value<S>::load(ra, voff + BB * u);
  }
  const __amdgpu_buffer_rsrc_t rl = span_rsrc(lslot + first, 4 * nb);
  P.ls = (int)__builtin_amdgcn_raw_buffer_load_b32(rl, 4 * lane, 0, 0);
  const int rv = r < 7 ? r : 6;
  if (BWD) {
    P.base = yl[7 * (size_t)T.row + rv];
    // D_i precedes the row's first U block; chunks other than the last read a U block
    // here, which they do not use
    P.D = Value<S>::load(span_rsrc(fac + 49 * (size_t)(T.first - 1), BB), voff);
  } else {
    P.base = (C)v[7 * (size_t)(T.vtx & 0x7fffffff) + rv];
  }
}

// ybuf_c: this lane's component column of the LDS slots (byte address of ybuf + c * sizeof(C));
// acc: the row's partial sums, carried from task to task while a row continues
template <typename C, int BWD, int MB>
__device__ __forceinline__ void task_run(const TaskMeta& T, const TaskData<C, MB>& P, const char* ybuf_c, C* ybuf,
                                         C* yl, double* __restrict__ z, C (&acc)[4], int r, int c) {
  const int nb = T.last - T.first;
  const int cc = c < 7 ? c : 6;
  if (!(T.flags & kTaskCont)) acc[0] = acc[1] = acc[2] = acc[3] = (C)0;
  // groups of eight blocks: the LDS reads of a group are issued together; blocks beyond
  // the range contribute A = 0 times a finite slot value.  Block b goes to acc[b % 4]:
  // four independent FMA chains.
#pragma unroll
  for (int g = 0; g < MB; g += 8) {
    if (g < nb) {
      C yv[8];
#pragma unroll
      for (int u = 0; u < 8 && g + u < MB; ++u)
        yv[u] = *(const C*)(ybuf_c + __builtin_amdgcn_readlane(P.ls, g + u));
#pragma unroll
      for (int u = 0; u < 8 && g + u < MB; ++u) acc[u & 3] = fma(P.A[g + u], yv[u], acc[u & 3]);
    }
  }
  if (T.flags & kTaskMore) return;
  // sum_c of row r of all blocks times the column values
  const C sum = sum8<C>((acc[0] + acc[1]) + (acc[2] + acc[3]));
  C out;
  if (!BWD) {
    out = P.base - sum;                                   // y_i = b_i - sum_k L_ik y_k
    if (c == 0 && r < 7) yl[7 * (size_t)T.row + r] = out;
  } else {
    const C t = P.base - sum;                             // y_i - sum_j U_ij x_j
    const C tc = __shfl(t, 8 * cc, 64);                   // component cc: lanes of row cc
    out = sum8<C>(P.D * tc);                              // x_i = D_i (...)
    if (c == 0 && r < 7 && T.vtx < 0) z[7 * (size_t)(T.vtx & 0x7fffffff) + r] = (double)out;
  }
  if (T.slot >= 0 && c == 0 && r < 7) ybuf[7 * T.slot + r] = out;
}

template <typename S, int BWD, int MB, int D>
__global__ void __launch_bounds__(64 * kSweepWaves) k_ilu_sweep(const int32_t* __restrict__ nphase,
                                                               const int32_t* __restrict__ wtask,
                                                               const int4* __restrict__ task,
                                                               const int4* __restrict__ aux,
                                                               const int32_t* __restrict__ lslot,
                                                               const S* __restrict__ fac,
                                                               const double* __restrict__ v,
                                                               typename Value<S>::C* yl, double* __restrict__ z,
                                                               int32_t* __restrict__ flags, int nslots,
                                                               int wait_limit) {
  using C = typename Value<S>::C;
  extern __shared__ double lds_d[];
  C* lds = (C*)lds_d;
  C* ybuf = lds;                               // [nslots][7]
  const int s = blockIdx.x;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r = lane >> 3, c = lane & 7;
  const int e = 7 * (r < 7 ? r : 6) + (c < 7 ? c : 6);   // block entry of the lane
  const int voff = (r < 7 && c < 7) ? (int)sizeof(S) * e : kOutside;
  const char* ybuf_c = (const char*)ybuf + sizeof(C) * (c < 7 ? c : 6);
  const int nL = nphase[s];
  const int tb = wtask[s * kSweepWaves + wave], te = wtask[s * kSweepWaves + wave + 1];
  // progress phases of the wavefronts: every row of wavefront w with a phase below prog[w]
  // is finished (its slot written, all its reads done)
  __shared__ int prog[kSweepWaves];
  int mine = te > tb ? __builtin_amdgcn_readfirstlane(aux[tb].w) : nL;  // the next row's phase
  if (lane == 0) prog[wave] = mine;
  // slots are read before their first write only through blocks with A = 0: keep them finite
  for (int t = threadIdx.x; t < 7 * nslots; t += 64 * kSweepWaves) ybuf[t] = (C)0;
  __syncthreads();
  int seen = 0;      // a lower bound of min_w prog[w] (the phases only grow)
  bool live = true;  // false once a wait has exceeded its bound
  // wait until every row of a phase below p is finished; the acquire fence keeps the slot
  // reads after the wait
  auto wait_phase = [&](int p) {
    if (p <= seen || !live) return;
    for (int spins = 0;; ++spins) {
      int m = nL;
#pragma unroll
      for (int w = 0; w < kSweepWaves; ++w)
        m = min(m, __hip_atomic_load(&prog[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
      seen = __builtin_amdgcn_readfirstlane(m);
      if (p <= seen) break;
      if (spins == wait_limit) {
        live = false;
        if (lane == 0) atomicOr(&flags[3], 1);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
  };
  C acc[4] = {(C)0, (C)0, (C)0, (C)0};
  if (te > tb) {
    // c0 holds tasks [cb, cb + 64) and c1 the next chunk; consecutive chunks overlap by
    // D - 1 tasks, so task t and the task t + D - 1 loaded with it always share c0 and c1
    // is touched only when it becomes c0, long after its load.
    constexpr int kStride = 64 - (D - 1);
    int cb = tb;
    TaskChunk c0 = load_chunk(task, aux, cb, te, lane);
    TaskChunk c1 = load_chunk(task, aux, cb + kStride, te, lane);
    TaskData<C, MB> buf[D];
    // tasks tb .. tb + D - 2 in flight before the first runs; the loop keeps D - 1 ahead
#pragma unroll
    for (int k = 0; k + 1 < D; ++k) {
      const int u = tb + k < te ? tb + k : te - 1;
      task_load<S, BWD, MB>(buf[k], chunk_get(c0, u - cb), lslot, fac, v, yl, lane, voff, r);
    }
    for (int t0 = tb; t0 < te; t0 += D) {
#pragma unroll
      for (int k = 0; k < D; ++k) {
        const int t = t0 + k;
        if (t < te && t + D - 1 - cb == 64) {  // the chunk at cb + kStride starts at task t
          c0 = c1;
          cb += kStride;
          c1 = load_chunk(task, aux, cb + kStride, te, lane);
        }
        if (t < te) {
          const TaskMeta T = chunk_get(c0, t - cb);
          wait_phase(T.phase);
          task_run<C, BWD, MB>(T, buf[k], ybuf_c, ybuf, yl, z, acc, r, c);
          // Release: when the next task belongs to a row of a later phase, this wavefront's
          // rows below that phase are finished; publish it (after the slot write and the
          // slot reads have completed) before the prefetch below and before any leading
          // task of that row, so that the rows waiting on it wait for neither.
          const int next_phase = t + 1 < te ? __builtin_amdgcn_readlane(c0.a.w, t + 1 - cb) : nL;
          if (next_phase > mine) {
            mine = next_phase;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
            if (lane == 0) __hip_atomic_store(&prog[wave], mine, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          }
        }
        // prefetch of task t + D - 1 into the set task t - 1 used (a fixed number of loads
        // per task, also past the end, so that every wait on the memory counter is exact)
        const int u = t + D - 1 < te ? t + D - 1 : te - 1;
        task_load<S, BWD, MB>(buf[(k + D - 1) % D], chunk_get(c0, u - cb), lslot, fac, v, yl, lane, voff, r);
      }
    }
  }
}

// yl_ws: the forward sweep's results, 7 values of the arithmetic type per local row (every
// one written before it is read); flags_ws: the four error flags (the sweeps raise [3])
template <typename S, int MB, int D>
static hipError_t launch_sweeps(fsi_solver* s, const S* facs, const double* v, double* z, void* yl_ws,
                                int32_t* flags_ws) {
  using C = typename Value<S>::C;
  constexpr int NT = 64 * kSweepWaves;
  const size_t lds = (size_t)s->h.nslots * 7 * sizeof(C);
  if (lds > 160 * 1024 - 64) return hipErrorInvalidConfiguration;  // 64 B for the progress phases
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)k_ilu_sweep<S, 0, MB, D>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e == hipSuccess)
      e = hipFuncSetAttribute((const void*)k_ilu_sweep<S, 1, MB, D>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
    if (e != hipSuccess) return e;
  }
  C* yl = (C*)yl_ws;
  FSI_PROF_LAUNCH(s, "ilu_fwd",
                  hipLaunchKernelGGL((k_ilu_sweep<S, 0, MB, D>), dim3(s->h.ns), dim3(NT), lds, s->stream,
                                     s->fwd_nphase, s->fwd_wtask, s->fwd_task, s->fwd_task_aux, s->lslot, facs, v, yl,
                                     z, flags_ws, s->h.nslots, s->wait_limit));
  FSI_PROF_LAUNCH(s, "ilu_bwd",
                  hipLaunchKernelGGL((k_ilu_sweep<S, 1, MB, D>), dim3(s->h.ns), dim3(NT), lds, s->stream,
                                     s->bwd_nphase, s->bwd_wtask, s->bwd_task, s->bwd_task_aux, s->lslot, facs, v, yl,
                                     z, flags_ws, s->h.nslots, s->wait_limit));
  return hipGetLastError();
}

template <typename S>
static hipError_t launch_sweeps_mb(fsi_solver* s, const S* facs, const double* v, double* z, void* yl_ws,
                                   int32_t* flags_ws) {
  switch (s->sweep_mb) {  // the candidates of kSweepPlanMB, each with its prefetch depth
    case 8: return launch_sweeps<S, 8, 6>(s, facs, v, z, yl_ws, flags_ws);
    case 16: return launch_sweeps<S, 16, 4>(s, facs, v, z, yl_ws, flags_ws);
    case 24: return launch_sweeps<S, 24, 3>(s, facs, v, z, yl_ws, flags_ws);
    case 32: return launch_sweeps<S, 32, 2>(s, facs, v, z, yl_ws, flags_ws);
    default: return hipErrorInvalidValue;
  }
}

// Blocks per sweep task (rows are split into tasks of at most this many blocks) and the
// matching kernels: the tasks in flight per wavefront shrink as tasks grow, keeping the
// prefetched blocks within the register file.
int sweep_task_blocks(int longest_part) { return longest_part <= 16 ? 16 : 24; }

hipError_t launch_pc_apply_ws(fsi_solver* s, const double* v, double* z, void* yl_ws, int32_t* flags_ws) {
  switch (s->opts.precision) {
    case FSI_PREC_FP64: return launch_sweeps_mb<double>(s, s->fac, v, z, yl_ws, flags_ws);
    case FSI_PREC_FP32: return launch_sweeps_mb<float>(s, (const float*)s->facs, v, z, yl_ws, flags_ws);
    case FSI_PREC_BF16: return launch_sweeps_mb<bf16_t>(s, (const bf16_t*)s->facs, v, z, yl_ws, flags_ws);
    case FSI_PREC_FP32_FACTOR: return launch_sweeps_mb<float>(s, s->fac32, v, z, yl_ws, flags_ws);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_pc_apply(fsi_solver* s, const double* v, double* z) {
  return launch_pc_apply_ws(s, v, z, s->ylocal, s->flags);
}

size_t pc_apply_ws_bytes(const fsi_solver* s) {
  return (size_t)s->R * 7 * (s->opts.precision == FSI_PREC_FP64 ? sizeof(double) : sizeof(float));
}

// Rounded factors for the mixed-precision sweeps, written in place over the FP64 factors:
// rounded value i (w = sizeof(S) bytes) goes to byte w*i of the same buffer.  The values are
// taken in chunks of kRoundChunk; each workgroup reads its whole chunk into registers before
// it writes any of it.  Chunk c's output covers FP64 entries [c*B*w/8, (c+1)*B*w/8), so a
// launch over chunks [a, 8a/w) writes only into chunks below a, all read by earlier launches
// on the same stream, and reads nothing that it writes.  Chunk 0 (which writes into itself)
// has a launch of its own.
constexpr int kRoundChunk = 256 * 8;

__device__ __forceinline__ void round_to(float* out, int64_t i, double x) { out[i] = (float)x; }
__device__ __forceinline__ void round_to(uint16_t* out, int64_t i, double x) {
  const uint32_t u = __float_as_uint((float)x);
  // round to nearest even on the 16 dropped bits; NaN stays NaN
  const uint32_t r = ((u & 0x7fffffffu) > 0x7f800000u) ? (u | 0x00400000u) : u + 0x7fffu + ((u >> 16) & 1u);
  out[i] = (uint16_t)(r >> 16);
}

template <typename S>
__global__ void __launch_bounds__(256) k_fac_round_inplace(int64_t n, int64_t c0, double* fac) {
  const int64_t base = (c0 + blockIdx.x) * (int64_t)kRoundChunk;
  double v[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int64_t i = base + 256 * u + threadIdx.x;
    v[u] = i < n ? fac[i] : 0.0;
  }
  __syncthreads();
  S* out = reinterpret_cast<S*>(fac);
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int64_t i = base + 256 * u + threadIdx.x;
    if (i < n) round_to(out, i, v[u]);
  }
}

template <typename S>
static hipError_t round_inplace(fsi_solver* s, int64_t n) {
  const int64_t nchunk = (n + kRoundChunk - 1) / kRoundChunk;
  const int64_t ratio = 8 / (int64_t)sizeof(S);
  hipLaunchKernelGGL(k_fac_round_inplace<S>, dim3(1), dim3(256), 0, s->stream, n, int64_t(0), s->fac);
  for (int64_t a = 1; a < nchunk;) {
    const int64_t b = std::min(nchunk, a * ratio);
    hipLaunchKernelGGL(k_fac_round_inplace<S>, dim3((unsigned)(b - a)), dim3(256), 0, s->stream, n, a, s->fac);
    a = b;
  }
  return hipGetLastError();
}

hipError_t launch_fac_round(fsi_solver* s) {
  const int64_t n = s->NB * 49;
  if (n == 0 || s->opts.precision == FSI_PREC_FP64 || s->opts.precision == FSI_PREC_FP32_FACTOR) return hipSuccess;
  return s->opts.precision == FSI_PREC_FP32 ? round_inplace<float>(s, n) : round_inplace<uint16_t>(s, n);
}

}  // namespace fsi
