// Vertex-patch additive Schwarz: one element-structured LOR V-cycle per patch
// (Sections 3.2-3.4), summed into z (eq. as).
//
// One wavefront per patch.  The ILU(0) sweeps in MDF order are a chain of
// dependency levels of a few rows each, so the kernel is built around latency:
//  * patch vectors stay in LDS (unpadded boxes); at the finest level only two
//    (the residual is re-gathered from global memory when needed), so several
//    patches share a CU;
//  * the wavefront synchronises with wave-scope fences only (no s_barrier,
//    no waits on outstanding global loads);
//  * each triangular sweep is stored in chunks of consecutive dependency
//    levels, at most one row per lane and chunk (a row with many couplings
//    takes a lane pair that adds its two partial sums), interleaved by lane
//    so that a chunk arrives in a few coalesced loads; chunk c+1 is loaded
//    into a second register buffer while the levels of chunk c run;
//  * in float64, residuals and prolongations take two rows per lane, so
//    that two stencil records or table lookups per lane are in flight; in
//    float32 one, which keeps the kernel at 111 registers and 14 patches
//    per CU (the LDS limit).
// Corrections of overlapping patches are added with FP64 atomics.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "lor_internal.h"

namespace lor {

namespace {


__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

template <int DIM>
struct Box {
  int m[3];   // unknowns per direction
  int lo[3];  // first level-grid index per direction
  int n;      // unknowns
};

// Box of the patch of vertex v at level k (recomputed instead of stored, so
// that nothing is indexed dynamically in private memory).
template <int DIM>
__device__ __forceinline__ Box<DIM> make_box(const PatchArgs &pa, const int *v, int k) {
  Box<DIM> b;
  const int s = pa.s[k];
  b.n = 1;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (d >= DIM) {
      b.m[d] = 1;
      b.lo[d] = 0;
      continue;
    }
    const int nn = pa.md.n[d];
    const int lo = v[d] > 0 ? (v[d] - 1) * s + 1 : 1;
    const int hi = v[d] < nn ? (v[d] + 1) * s - 1 : nn * s - 1;
    b.lo[d] = lo;
    b.m[d] = max(hi - lo + 1, 0);
    b.n *= b.m[d];
  }
  return b;
}

template <int DIM>
__device__ inline int64_t level_gidx(const Box<DIM> &bx, int i, const int *lng) {
  const int ix = i % bx.m[0], iy = (i / bx.m[0]) % bx.m[1],
            iz = DIM == 3 ? i / (bx.m[0] * bx.m[1]) : 0;
  return int64_t(bx.lo[0] + ix) +
         int64_t(lng[0]) * (int64_t(bx.lo[1] + iy) + (DIM == 3 ? int64_t(lng[1]) * (bx.lo[2] + iz) : 0));
}

// Coordinates of row i of a box and of the rows after it at a fixed stride,
// advanced without a division per row (one division when the walk starts).
template <int DIM>
struct Walk {
  int x, y, z;     // current row
  int dx, dy, dz;  // the stride in coordinates (dx < m0, dy < m1)
  int m0, m1;
  Walk() = default;
  __device__ __forceinline__ Walk(const Box<DIM> &bx, int i, int stride) {
    m0 = max(bx.m[0], 1);
    m1 = max(bx.m[1], 1);
    x = i % m0;
    const int t = i / m0;
    y = t % m1;
    z = t / m1;
    dx = stride % m0;
    const int u = stride / m0;
    dy = u % m1;
    dz = u / m1;
  }
  __device__ __forceinline__ void step() {
    x += dx;
    const bool cx = x >= m0;
    x = cx ? x - m0 : x;
    y += dy + (cx ? 1 : 0);
    const bool cy = y >= m1;
    y = cy ? y - m1 : y;
    z += dz + (cy ? 1 : 0);
  }
};

// level-grid index of the walk's current row
template <int DIM>
__device__ __forceinline__ int64_t walk_gidx(const Box<DIM> &bx, const Walk<DIM> &w, const int *lng) {
  const int t = (bx.lo[1] + w.y) + (DIM == 3 ? lng[1] * (bx.lo[2] + w.z) : 0);
  return int64_t(bx.lo[0] + w.x) + int64_t(lng[0]) * t;
}

// index of the walk's current row (a level-0 box) in the global vectors
template <int DIM>
__device__ __forceinline__ int64_t walk_uidx(const Box<DIM> &bx, const Walk<DIM> &w, const MeshDims &md) {
  const int ox = md.dirichlet ? 1 : 0;
  const int t = (bx.lo[1] + w.y - ox) + (DIM == 3 ? md.nu[1] * (bx.lo[2] + w.z - ox) : 0);
  return int64_t(bx.lo[0] + w.x - ox) + int64_t(md.nu[0]) * t;
}

// Partition-of-unity weight 1/c(i) of the walk's current row (a level-0
// box): a level-0 grid coordinate g lies in the patches of the vertices
// around it, one in a direction where g is on a vertex line (g a multiple of
// p) and two elsewhere, so c = prod_d c_d.
template <int DIM>
__device__ __forceinline__ double pou_weight(const Box<DIM> &bx, const Walk<DIM> &w, int p) {
  const int g[3] = {bx.lo[0] + w.x, bx.lo[1] + w.y, DIM == 3 ? bx.lo[2] + w.z : 0};
  double c = 1.0;
  for (int d = 0; d < DIM; ++d) c *= (g[d] % p == 0) ? 1.0 : 0.5;
  return c;
}

// LDS layout of one patch (values of T):
//   X_0 | B_0 (warm start only) | R_0 | B_1
// and, inside R_0's space, X_1, R_1, then X_k, B_k, R_k for k >= 2: R_0 is
// dead from the restriction to level 1 (which reads R_0 and writes B_1, kept
// apart) until the level-0 residual after the prolongation from level 1.
// Without a warm start the level-0 right side is the global residual.
// which: 0 = X, 1 = B, 2 = R.
template <int DIM, typename T, bool WARM>
__device__ __forceinline__ T *lds_vec(T *lds, const PatchArgs &pa, const int *v, int k, int which) {
  const int n0 = make_box<DIM>(pa, v, 0).n;
  T *R0 = lds + (WARM ? 2 : 1) * n0;
  if (k == 0) return which == 0 ? lds : (which == 2 ? R0 : (WARM ? lds + n0 : nullptr));
  const int n1 = make_box<DIM>(pa, v, 1).n;
  if (k == 1) return which == 0 ? R0 : (which == 1 ? R0 + n0 : R0 + n1);
  int off = 2 * n1;
  for (int q = 2; q < k; ++q) off += 3 * make_box<DIM>(pa, v, q).n;
  return R0 + off + which * make_box<DIM>(pa, v, k).n;
}

// ---------------------------------------------------------------- sweeps
// A sweep block (layout at kChunkLanes) is consumed chunk by chunk from two
// register buffers: wait for chunk c, issue the coalesced loads of chunk c+1
// into the other buffer, then run the dependency levels of chunk c from
// registers and LDS.  The only wait on global memory is the one before new
// loads are issued, so the loads of a chunk overlap a whole chunk of levels.

// Word k of a register record (k is a constant after unrolling, so the
// record stays in registers).
template <int QM>
__device__ __forceinline__ uint32_t wget(const uint4 (&R)[QM], int k) {
  const uint4 q = R[k >> 2];
  switch (k & 3) {
    case 0: return q.x;
    case 1: return q.y;
    case 2: return q.z;
    default: return q.w;
  }
}
template <typename T, int QM>
__device__ __forceinline__ T word_get(const uint4 (&R)[QM], int b) {
  if constexpr (sizeof(T) == 4)
    return __uint_as_float(wget(R, b));
  else
    return __hiloint2double(int(wget(R, b + 1)), int(wget(R, b)));
}

// Value of lane l ^ 1 (DPP quad permutation [1, 0, 3, 2]; every lane active).
__device__ __forceinline__ float pair_swap(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0xB1, 0xF, 0xF, false));
}
__device__ __forceinline__ double pair_swap(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), 0xB1, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), 0xB1, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ void wait_vm() { __builtin_amdgcn_s_waitcnt(0x0F70); }  // vmcnt(0)
__device__ __forceinline__ void wait_lds() { __builtin_amdgcn_s_waitcnt(0xC07F); }  // lgkmcnt(0)

// Loads this lane's record of a chunk (myq quads).  The loads are branch
// free: quads the lane does not need read a zero quad of the block header, so
// the data goes straight into the record registers and nothing waits for it
// until the chunk is used.
template <typename T, bool FWD, int QM>
__device__ __forceinline__ void load_chunk(uint4 (&R)[QM], const uint4 *src, int myq, const uint4 *zero) {
#pragma unroll
  for (int q = 0; q < QM; ++q) {
    const uint4 *a = q < myq ? src + (q * 64 + int(threadIdx.x)) : zero;
    R[q] = *a;
  }
}

// The steps of one chunk with NPP coupling pairs per lane record: the
// chunk's widest record (records with fewer couplings have zero padding
// couplings that read the row itself), so a chunk of narrow rows costs fewer
// LDS reads and FMAs.  SPLIT: the chunk holds rows split over a lane pair; the
// second lane of a pair starts from zero, and the first adds the pair's
// partial sum.  The neighbours' LDS indices come from the record's slot mask
// and the level box's slot table, once per chunk.
template <typename T, bool FWD, int QM, int NPP, bool SPLIT>
__device__ __forceinline__ void run_steps(const uint4 (&R)[QM], T *Y, const short *tab, int nsteps,
                                          int mystep, int row, bool second, bool paired) {
  constexpr int H = sweep_head_words<T>(FWD), SZ = int(sizeof(T)) / 4;
  int nb[2 * NPP + 1];
  {
    uint32_t m = wget(R, H);
    // table reads for every coupling slot first, one LDS wait for all of them
#pragma unroll
    for (int k = 0; k < 2 * NPP; ++k) {
      const uint32_t sl = m ? uint32_t(__builtin_ctz(m)) : 27u;  // 27: padding, offset 0
      m &= m - 1;
      nb[k] = tab[sl];
    }
#pragma unroll
    for (int k = 0; k < 2 * NPP; ++k) nb[k] += row;
  }
  for (int s = 0; s < nsteps; ++s) {
    T part = T(0);
    if (mystep == s) {
      T acc0 = FWD ? Y[row] : Y[row] * word_get<T, QM>(R, 1);
      if (SPLIT) acc0 = second ? T(0) : acc0;
      T acc1 = T(0);
      // all LDS reads are issued before the FMAs, with no branch between them
      // (padding couplings have zero values and read the row itself), so a
      // step costs one LDS round trip
      T y[2 * NPP + 2];
#pragma unroll
      for (int k = 0; k < 2 * NPP; ++k) y[k] = Y[nb[k]];
      // one wait for all of them (fewer instructions per step than a wait
      // before every FMA); the scheduling barriers keep it in place
      __builtin_amdgcn_sched_barrier(0);
      wait_lds();
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int p = 0; p < NPP; ++p) {
        acc0 -= word_get<T, QM>(R, H + 1 + (2 * p) * SZ) * y[2 * p];
        acc1 -= word_get<T, QM>(R, H + 1 + (2 * p + 1) * SZ) * y[2 * p + 1];
      }
      if (SPLIT)
        part = acc0 + acc1;
      else
        Y[row] = acc0 + acc1;
    }
    if (SPLIT) {
      const T other = pair_swap(part);
      if (mystep == s && !second) Y[row] = paired ? part + other : part;
    }
    wave_sync();
  }
}

template <typename T, bool FWD, int QM, bool SPLIT>
__device__ __forceinline__ void run_chunk_w(const uint4 (&R)[QM], T *Y, const short *tab, int npairs,
                                            int nsteps, int mystep, int row, bool second, bool paired) {
  switch (npairs) {
    case 0: run_steps<T, FWD, QM, 0, SPLIT>(R, Y, tab, nsteps, mystep, row, second, paired); break;
    case 1: run_steps<T, FWD, QM, 1, SPLIT>(R, Y, tab, nsteps, mystep, row, second, paired); break;
    case 2: run_steps<T, FWD, QM, 2, SPLIT>(R, Y, tab, nsteps, mystep, row, second, paired); break;
    case 3: run_steps<T, FWD, QM, 3, SPLIT>(R, Y, tab, nsteps, mystep, row, second, paired); break;
    case 4: run_steps<T, FWD, QM, 4, SPLIT>(R, Y, tab, nsteps, mystep, row, second, paired); break;
    case 5: run_steps<T, FWD, QM, 5, SPLIT>(R, Y, tab, nsteps, mystep, row, second, paired); break;
    case 6: run_steps<T, FWD, QM, 6, SPLIT>(R, Y, tab, nsteps, mystep, row, second, paired); break;
    default: run_steps<T, FWD, QM, kLaneCouplings / 2, SPLIT>(R, Y, tab, nsteps, mystep, row, second, paired); break;
  }
}

template <typename T, bool FWD, int QM>
__device__ __forceinline__ void run_chunk(const uint4 (&R)[QM], T *Y, const short *tab, uint32_t hdr) {
  const int nsteps = (hdr >> 8) & 0xFF;
  const int npairs = int((hdr >> 16) & 0xFF) / 2;  // the chunk's widest record, in pairs
  const uint32_t d0 = R[0].x;
  const int mystep = (d0 & kSweepValid) ? int((d0 >> 16) & 0x3F) : -1;
  const int row = int(d0 & 0xFFFF);
  if (hdr & kChunkSplit)
    run_chunk_w<T, FWD, QM, true>(R, Y, tab, npairs, nsteps, mystep, row, (d0 & kSweepSecond) != 0,
                                  (d0 & kSweepPaired) != 0);
  else
    run_chunk_w<T, FWD, QM, false>(R, Y, tab, npairs, nsteps, mystep, row, false, false);
}

// Slot table of a level box with extents m0 x m1 (x ...): entry s the LDS
// offset of stencil slot s (x fastest: (s%3-1) + m0 ((s/3)%3-1) + m0 m1
// (s/9-1)), entry 27 zero (padding couplings).
template <int DIM>
__device__ __forceinline__ void slot_table(short *tab, int m0, int m1) {
  const int s = int(threadIdx.x);
  if (s < 28) {
    int o = 0;
    if (s < (DIM == 3 ? 27 : 9)) o = (s % 3 - 1) + m0 * ((s / 3) % 3 - 1) + (DIM == 3 ? m0 * m1 * (s / 9 - 1) : 0);
    tab[s] = short(o);
  }
  wave_sync();
}

// forward:  w_i = y_i - sum_{earlier m} l_im w_m
// backward: y_i = w_i / D_i - sum_{later m} l_mi y_m       (both in place on Y)
template <typename T, bool FWD>
__device__ __forceinline__ void sweep(T *Y, const char *blk, const short *tab) {
  constexpr int QM = sweep_quads<T>(FWD, kLaneCouplings);
  const int nch = *reinterpret_cast<const int *>(blk);
  uint32_t hdr = reinterpret_cast<const uint32_t *>(blk)[1];
  const int lane = threadIdx.x;
  auto nextq = [&](uint32_t w0) { return lane == 63 ? 1 : int((w0 >> 22) & 0x1F); };
  const uint4 *src = reinterpret_cast<const uint4 *>(blk + kSweepHeader);
  const uint4 *zero = reinterpret_cast<const uint4 *>(blk + kSweepZero);
  uint4 A[QM], B[QM];
  load_chunk<T, FWD, QM>(A, src, int(reinterpret_cast<const unsigned char *>(blk)[16 + lane]), zero);
  src += int(hdr & 0xFF) * 64;
  for (int c = 0; c < nch; c += 2) {
    wait_vm();
    const uint32_t h1 = __builtin_amdgcn_readlane(A[0].x, 63);
    if (c + 1 < nch) {
      load_chunk<T, FWD, QM>(B, src, nextq(A[0].x), zero);
      src += int(h1 & 0xFF) * 64;
    }
    run_chunk<T, FWD, QM>(A, Y, tab, hdr);
    if (c + 1 >= nch) break;
    wait_vm();
    const uint32_t h2 = __builtin_amdgcn_readlane(B[0].x, 63);
    if (c + 2 < nch) {
      load_chunk<T, FWD, QM>(A, src, nextq(B[0].x), zero);
      src += int(h2 & 0xFF) * 64;
    }
    run_chunk<T, FWD, QM>(B, Y, tab, h1);
    hdr = h2;
  }
}

// A point's stencil record with 16-byte loads (records are 16-byte aligned):
// a[s] = coefficient of slot s; in the symmetric half-records (double) only
// slots C.. are filled.
template <int DIM, typename ST>
__device__ __forceinline__ void load_rec(const ST *__restrict__ rec, ST *a) {
  constexpr int W = rec_width<DIM, ST>(), NS = DIM == 3 ? 27 : 9, C = NS / 2;
  constexpr int PER = 16 / int(sizeof(ST));  // values per 16-byte load
  ST v[W];
#pragma unroll
  for (int q = 0; q < W / PER; ++q) {
    if constexpr (sizeof(ST) == 4) {
      const float4 t = reinterpret_cast<const float4 *>(rec)[q];
      v[4 * q] = t.x;
      v[4 * q + 1] = t.y;
      v[4 * q + 2] = t.z;
      v[4 * q + 3] = t.w;
    } else {
      const double2 t = reinterpret_cast<const double2 *>(rec)[q];
      v[2 * q] = t.x;
      v[2 * q + 1] = t.y;
    }
  }
  if constexpr (sizeof(ST) == 4) {
#pragma unroll
    for (int s = 0; s < NS; ++s) a[s] = v[s];
  } else {
#pragma unroll
    for (int j = 0; j <= C; ++j) a[C + j] = v[j];
  }
}

// Neighbour s of a row whose coordinates satisfy the six edge tests
// (xl: x > 0, xh: x < m0 - 1, ...) lies inside the box.
template <int DIM>
__device__ __forceinline__ bool nb_inside(int s, bool xl, bool xh, bool yl, bool yh, bool zl, bool zh) {
  const int sx = s % 3 - 1, sy = (s / 3) % 3 - 1, sz = DIM == 3 ? s / 9 - 1 : 0;
  return (sx < 0 ? xl : (sx > 0 ? xh : true)) && (sy < 0 ? yl : (sy > 0 ? yh : true)) &&
         (sz < 0 ? zl : (sz > 0 ? zh : true));
}

// R = B - A X on one level from full records (float): each row reads its own
// record only.  GB: the right side is the global residual (finest level)
// instead of B in LDS.  Row coordinates come from a walk.
template <int DIM, typename T, typename ST, bool GB>
__device__ __forceinline__ void residual_full(T *R, const T *B, const T *X, const Box<DIM> &bx,
                                              const ST *__restrict__ st, const int *lng,
                                              const double *__restrict__ rglob, const MeshDims &md) {
  constexpr int NS = DIM == 3 ? 27 : 9, W = rec_width<DIM, ST>();
  // rows per lane and pass: two stencil records in flight per lane in float64
  // (its patches are few per CU, LDS-bound); one in float32, whose 111
  // registers let a fourth wavefront per SIMD in (14 patches per CU, 12 with
  // two rows: the added occupancy wins since the sweep records were sorted)
  constexpr int RB = sizeof(T) == 4 ? 1 : 2;
  const int mx = bx.m[0], my = bx.m[1], mz = bx.m[2];
  Walk<DIM> w[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) w[r] = Walk<DIM>(bx, threadIdx.x + 64 * r, 64 * RB);
  for (int i0 = threadIdx.x; i0 < bx.n; i0 += 64 * RB) {
    ST a[RB][NS];
    T acc[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      // a row past the end reads row i0's data (always a row of the box)
      const bool live = i0 + 64 * r < bx.n;
      const Walk<DIM> &wr = live ? w[r] : w[0];
      const int64_t g = walk_gidx<DIM>(bx, wr, lng);
      if (GB)
        acc[r] = T(rglob[walk_uidx<DIM>(bx, wr, md)]);
      else
        acc[r] = B[live ? i0 + 64 * r : i0];
      load_rec<DIM, ST>(st + g * W, a[r]);
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const int i = i0 + 64 * r;
      const bool live = i < bx.n;
      const bool xl = w[r].x > 0, xh = w[r].x < mx - 1, yl = w[r].y > 0, yh = w[r].y < my - 1,
                 zl = w[r].z > 0, zh = w[r].z < mz - 1;
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int sx = s % 3 - 1, sy = (s / 3) % 3 - 1, sz = DIM == 3 ? s / 9 - 1 : 0;
        const int off = sx + mx * (sy + my * sz);
        const bool in = live && nb_inside<DIM>(s, xl, xh, yl, yh, zl, zh);
        acc[r] -= (in ? T(a[r][s]) : T(0)) * X[in ? i + off : i0];
      }
      if (live) R[i] = acc[r];
      w[r].step();
    }
  }
  wave_sync();
}

template <int DIM, typename T, typename ST, bool GB>
__device__ __forceinline__ void residual_scatter(T *R, const T *B, const T *X, const Box<DIM> &bx,
                                                 const ST *__restrict__ st, const int *lng,
                                                 const double *__restrict__ rglob, const MeshDims &md) {
  // Each row reads only its own record (centre and forward half):
  //   R[i]       = b_i - a(i,C) X[i] - sum_{s > C} a(i,s) X[i + o_s]
  //   R[i + o_s] -= a(i,s) X[i]   (the neighbour's backward coupling, equal
  //                                to a(i,s) by symmetry)
  // the second kind by LDS atomics into R, cleared first.
  constexpr int NS = DIM == 3 ? 27 : 9, C = NS / 2, W = rec_width<DIM, ST>();
  constexpr int RB = sizeof(T) == 4 ? 1 : 2;
  const int mx = bx.m[0], my = bx.m[1], mz = bx.m[2];
  for (int i = threadIdx.x; i < bx.n; i += 64) R[i] = T(0);
  wave_sync();
  Walk<DIM> w[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) w[r] = Walk<DIM>(bx, threadIdx.x + 64 * r, 64 * RB);
  for (int i0 = threadIdx.x; i0 < bx.n; i0 += 64 * RB) {
    ST a[RB][NS];
    T acc[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const bool live = i0 + 64 * r < bx.n;
      const Walk<DIM> &wr = live ? w[r] : w[0];
      const int64_t g = walk_gidx<DIM>(bx, wr, lng);
      if (GB)
        acc[r] = T(rglob[walk_uidx<DIM>(bx, wr, md)]);
      else
        acc[r] = B[live ? i0 + 64 * r : i0];
      load_rec<DIM, ST>(st + g * W, a[r]);
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const int i = i0 + 64 * r;
      const bool live = i < bx.n;
      const bool xl = w[r].x > 0, xh = w[r].x < mx - 1, yl = w[r].y > 0, yh = w[r].y < my - 1,
                 zl = w[r].z > 0, zh = w[r].z < mz - 1;
      const int ic = live ? i : i0;
      const T xi = X[ic];
      acc[r] -= T(a[r][C]) * xi;
#pragma unroll
      for (int s = C + 1; s < NS; ++s) {
        const int sx = s % 3 - 1, sy = (s / 3) % 3 - 1, sz = DIM == 3 ? s / 9 - 1 : 0;
        const int off = sx + mx * (sy + my * sz);
        const bool in = live && nb_inside<DIM>(s, xl, xh, yl, yh, zl, zh);
        const int jn = in ? i + off : i0;
        const T aij = in ? T(a[r][s]) : T(0);
        acc[r] -= aij * X[jn];
        if (in) atomicAdd(R + jn, -aij * xi);
      }
      if (live) atomicAdd(R + i, acc[r]);
      w[r].step();
    }
  }
  wave_sync();
}

// R = B - A X on one level of a patch: from full records in single precision,
// from symmetric half-records with LDS atomics in double precision (twice the
// bytes per coefficient: the half-record keeps a row's stencil in one
// 128-byte line).  Both read one line per row.
template <int DIM, typename T, typename ST, bool GB>
__device__ __forceinline__ void residual(T *R, const T *B, const T *X, const Box<DIM> &bx,
                                         const ST *__restrict__ st, const int *lng,
                                         const double *__restrict__ rglob, const MeshDims &md) {
  if constexpr (sizeof(ST) == 8)
    residual_scatter<DIM, T, ST, GB>(R, B, X, bx, st, lng, rglob, md);
  else
    residual_full<DIM, T, ST, GB>(R, B, X, bx, st, lng, rglob, md);
}

// LDS values per patch: the largest patch's, plus its level-0 right side
// with a warm start
template <int DIM, bool WARM>
__host__ __device__ inline size_t lds_values(const PatchArgs &pa) {
  size_t n0 = 1;
  for (int d = 0; d < DIM; ++d) n0 *= size_t(2 * pa.s[0] - 1);
  return size_t(pa.lds_total) + (WARM ? n0 : 0);
}

// bytes of the slot table after the patch vectors (28 int16 entries)
constexpr int kSlotTableBytes = 64;

// One wavefront per patch.  Modes: scatter-add the correction into z (the
// preconditioner); write it into the patch grid (dense, training data); or,
// with WARM, start from a prediction y_j of the patch solve (patch-grid
// values wy[block][G^d] times dscale[block], patches jfirst + block) and
// scatter y_j + V_j(r_j - A_j y_j).
template <bool JOBS>
struct PatchArg {
  using type = PatchArgs;
};
template <>
struct PatchArg<true> {
  using type = PatchJobs;
};
__device__ __forceinline__ const PatchArgs &job_args(const PatchArgs &a, int) { return a; }
__device__ __forceinline__ const PatchArgs &job_args(const PatchJobs &a, int k) { return a.p[k]; }

// With JOBS, the launch carries several problems: the block first finds its
// problem from the block ranges, then proceeds as in a launch of that
// problem alone.
template <int DIM, typename T, typename ST, int W, bool WARM, bool JOBS = false>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_patch_vcycle(typename PatchArg<JOBS>::type arg, const double *__restrict__ r_in,
                                                     double *__restrict__ z_in, const double *flag_in,
                                                     float *__restrict__ dense,
                                                     const double *__restrict__ dscale,
                                                     const float *__restrict__ wy, int jfirst) {
  int job = 0, blk = int(blockIdx.x);
  if constexpr (JOBS) {
    while (job + 1 < arg.njobs && blk >= arg.block0[job + 1]) ++job;
    blk -= arg.block0[job];
  }
  const PatchArgs &pa = job_args(arg, job);
  const double *__restrict__ r = r_in;
  double *__restrict__ z = z_in;
  const double *flag = flag_in;
  int slot = blk;  // the block's place in the launch order
  if (!WARM && pa.nrhs > 0) {
    // several right-hand sides: the blocks of one patch sit 8 apart (same XCD)
    const int b = blk, t = b >> 3, k = t % pa.nrhs;
    slot = (t / pa.nrhs) * 8 + (b & 7);
    if (slot >= pa.nv[0] * pa.nv[1] * (DIM == 3 ? pa.nv[2] : 1)) return;
    r = pa.rs[k];
    z = pa.zs[k];
    flag = pa.flags[k];
  }
  if (flag && flag[S_DONE] != 0.0) return;
  extern __shared__ __align__(16) char lds_raw[];
  T *lds = reinterpret_cast<T *>(lds_raw);
  short *tab = reinterpret_cast<short *>(lds_raw + lds_values<DIM, WARM>(pa) * sizeof(T));
  int j = jfirst + slot;
  if (!WARM && pa.perm) j = pa.perm[j];
  if (pa.color >= 0) {
    // the patches of one vertex-parity class: their level-0 boxes are
    // disjoint, so their corrections can be added without atomics
    int nvc[3], c[3];
    for (int d = 0; d < 3; ++d) {
      c[d] = (pa.color >> d) & 1;
      nvc[d] = d < DIM ? (pa.nv[d] - c[d] + 1) / 2 : 1;
    }
    const int i = blk;
    const int vx = 2 * (i % nvc[0]) + c[0], vy = 2 * ((i / nvc[0]) % nvc[1]) + c[1],
              vz = DIM == 3 ? 2 * (i / (nvc[0] * nvc[1])) + c[2] : 0;
    j = vx + pa.nv[0] * (vy + pa.nv[1] * vz);
  }
  const int L = pa.nlev;
  const MeshDims &md = pa.md;
  const int v[3] = {j % pa.nv[0], (j / pa.nv[0]) % pa.nv[1],
                    DIM == 3 ? j / (pa.nv[0] * pa.nv[1]) : 0};
  int typ[3] = {1, 1, 1};
  for (int d = 0; d < DIM; ++d) typ[d] = v[d] == 0 ? 0 : (v[d] == md.n[d] ? 2 : 1);
  const Box<DIM> b0 = make_box<DIM>(pa, v, 0);
  if (b0.n <= 0) return;
  {
    const int tot = (WARM ? 3 : 2) * b0.n + (L > 1 ? make_box<DIM>(pa, v, 1).n : 0);
    for (int i = threadIdx.x; i < tot; i += 64) lds[i] = T(0);
  }
  wave_sync();
  // patch-grid index of a level-0 row: grid point g_d = node - (v_d p - p + 1)
  auto grid_q = [&](const Walk<DIM> &w) {
    const int s0 = pa.s[0], G = 2 * s0 - 1;
    const int gx = w.x + b0.lo[0] - (v[0] * s0 - s0 + 1), gy = w.y + b0.lo[1] - (v[1] * s0 - s0 + 1),
              gz = DIM == 3 ? w.z + b0.lo[2] - (v[2] * s0 - s0 + 1) : 0;
    return gx + G * (gy + G * gz);
  };
  int G3 = 1;
  for (int d = 0; d < DIM; ++d) G3 *= 2 * pa.s[0] - 1;
  if (WARM) {
    // X_0 = y_j, then the level-0 right side B_0 = r_j - A_j y_j
    T *X0 = lds_vec<DIM, T, WARM>(lds, pa, v, 0, 0);
    T *B0 = lds_vec<DIM, T, WARM>(lds, pa, v, 0, 1);
    const T sc = T(dscale[blockIdx.x]);
    const float *yj = wy + int64_t(blockIdx.x) * G3;
    Walk<DIM> w(b0, threadIdx.x, 64);
    for (int i = threadIdx.x; i < b0.n; i += 64, w.step()) X0[i] = T(yj[grid_q(w)]) * sc;
    wave_sync();
    residual<DIM, T, ST, true>(B0, nullptr, X0, b0, reinterpret_cast<const ST *>(pa.stencil[0]), pa.lng[0], r, md);
  } else {
  // pre-smoothing input: X_0 = r restricted to the patch
  {
    T *X0 = lds_vec<DIM, T, WARM>(lds, pa, v, 0, 0);
    // batched: 8 loads in flight per lane (rows past the end read row i0,
    // their store is skipped)
    Walk<DIM> w(b0, threadIdx.x, 64);
    for (int i0 = threadIdx.x; i0 < b0.n; i0 += 64 * 8) {
      int64_t u[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        u[q] = i0 + 64 * q < b0.n ? walk_uidx<DIM>(b0, w, md) : u[0];
        w.step();
      }
      T t[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) t[q] = T(r[u[q]]);
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (i0 + 64 * q < b0.n) X0[i0 + 64 * q] = t[q];
    }
  }
  wave_sync();
  }

  const int nf = L - 1;
  const int64_t fbase = int64_t(j) * (nf > 0 ? nf : 1);
  const ST *const *stn = reinterpret_cast<const ST *const *>(pa.stencil);
  // ---------------- down
  for (int k = 0; k < nf; ++k) {
    const Box<DIM> fb = make_box<DIM>(pa, v, k);
    if (fb.n <= 0) break;
    T *Xk = lds_vec<DIM, T, WARM>(lds, pa, v, k, 0);
    T *Bk = (k > 0 || WARM) ? lds_vec<DIM, T, WARM>(lds, pa, v, k, 1) : nullptr;
    T *Rk = lds_vec<DIM, T, WARM>(lds, pa, v, k, 2);
    const char *bf = pa.fac + pa.fac_off[2 * (fbase + k)];
    const char *bb = pa.fac + pa.fac_off[2 * (fbase + k) + 1];
    if (k > 0 || WARM) {
      for (int i = threadIdx.x; i < fb.n; i += 64) Xk[i] = Bk[i];
      wave_sync();
    }
    slot_table<DIM>(tab, fb.m[0], fb.m[1]);
    sweep<T, true>(Xk, bf, tab);
    sweep<T, false>(Xk, bb, tab);
    if (k == 0 && !WARM)
      residual<DIM, T, ST, true>(Rk, Bk, Xk, fb, stn[k], pa.lng[k], r, md);
    else
      residual<DIM, T, ST, false>(Rk, Bk, Xk, fb, stn[k], pa.lng[k], r, md);
    const Box<DIM> cb = make_box<DIM>(pa, v, k + 1);
    if (cb.n > 0) {
      T *Bc = lds_vec<DIM, T, WARM>(lds, pa, v, k + 1, 1);
      const XferTab *tb0 = &pa.xfer[k * 3 + typ[0]];
      const XferTab *tb1 = &pa.xfer[k * 3 + typ[1]];
      const XferTab *tb2 = &pa.xfer[k * 3 + typ[DIM - 1]];
      Walk<DIM> wc(cb, threadIdx.x, 64);
      for (int i = threadIdx.x; i < cb.n; i += 64, wc.step()) {
        const int ci[3] = {wc.x, wc.y, DIM == 3 ? wc.z : 0};
        // fixed 3 x 3 (x 3) gather, absent entries have weight 0 and index 0:
        // every table load and LDS read is issued up front
        int fx[3], fy[3], fz[3];
        T wx[3], wy[3], wz[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          fx[a] = tb0->rf[ci[0]][a];
          wx[a] = T(tb0->rw[ci[0]][a]);
          fy[a] = tb1->rf[ci[1]][a];
          wy[a] = T(tb1->rw[ci[1]][a]);
          fz[a] = DIM == 3 ? tb2->rf[ci[2]][a] : 0;
          wz[a] = DIM == 3 ? T(tb2->rw[ci[2]][a]) : T(a == 0 ? 1 : 0);
        }
        T acc = T(0);
#pragma unroll
        for (int c = 0; c < (DIM == 3 ? 3 : 1); ++c)
#pragma unroll
          for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int a = 0; a < 3; ++a)
              acc += wx[a] * wy[b] * wz[c] * Rk[fx[a] + fb.m[0] * (fy[b] + fb.m[1] * fz[c])];
        Bc[i] = acc;
      }
      wave_sync();
    }
  }
  // ---------------- coarsest level: exact (at most one unknown)
  {
    const int kc = L - 1;
    const Box<DIM> bc = make_box<DIM>(pa, v, kc);
    if (bc.n == 1 && threadIdx.x == 0) {
      const int64_t g = level_gidx<DIM>(bc, 0, pa.lng[kc]);
      constexpr int C = DIM == 3 ? 13 : 4;
      T *Xc = lds_vec<DIM, T, WARM>(lds, pa, v, kc, 0);
      const T rhs = (kc == 0 && !WARM) ? Xc[0] : lds_vec<DIM, T, WARM>(lds, pa, v, kc, 1)[0];
      Xc[0] = rhs / T(stn[kc][g * rec_width<DIM, ST>() + rec_centre<DIM, ST>()]);
    }
    wave_sync();
  }
  // ---------------- up
  for (int k = nf - 1; k >= 0; --k) {
    const Box<DIM> fb = make_box<DIM>(pa, v, k);
    if (fb.n <= 0) continue;
    T *Xk = lds_vec<DIM, T, WARM>(lds, pa, v, k, 0);
    T *Bk = (k > 0 || WARM) ? lds_vec<DIM, T, WARM>(lds, pa, v, k, 1) : nullptr;
    T *Rk = lds_vec<DIM, T, WARM>(lds, pa, v, k, 2);
    const char *bf = pa.fac + pa.fac_off[2 * (fbase + k)];
    const char *bb = pa.fac + pa.fac_off[2 * (fbase + k) + 1];
    const Box<DIM> cb = make_box<DIM>(pa, v, k + 1);
    if (cb.n > 0) {
      const T *Xc = lds_vec<DIM, T, WARM>(lds, pa, v, k + 1, 0);
      const XferTab *tb0 = &pa.xfer[k * 3 + typ[0]];
      const XferTab *tb1 = &pa.xfer[k * 3 + typ[1]];
      const XferTab *tb2 = &pa.xfer[k * 3 + typ[DIM - 1]];
      // PB rows per lane and iteration (as the residual's RB); a row past
      // the end uses row i0's coordinates, its store is skipped
      constexpr int PB = sizeof(T) == 4 ? 1 : 2;
      Walk<DIM> wf[PB];
#pragma unroll
      for (int r = 0; r < PB; ++r) wf[r] = Walk<DIM>(fb, threadIdx.x + 64 * r, 64 * PB);
      for (int i0 = threadIdx.x; i0 < fb.n; i0 += 64 * PB) {
        // fixed 2 x 2 (x 2) gather; sources on the patch boundary get weight 0
        int cx[PB][2], cy[PB][2], cz[PB][2];
        T wx[PB][2], wy[PB][2], wz[PB][2];
#pragma unroll
        for (int r = 0; r < PB; ++r) {
          const Walk<DIM> &wr = i0 + 64 * r < fb.n ? wf[r] : wf[0];
          const int fi[3] = {wr.x, wr.y, DIM == 3 ? wr.z : 0};
#pragma unroll
          for (int a = 0; a < 2; ++a) {
            cx[r][a] = tb0->pc[fi[0]][a];
            wx[r][a] = T(tb0->pw[fi[0]][a]);
            cy[r][a] = tb1->pc[fi[1]][a];
            wy[r][a] = T(tb1->pw[fi[1]][a]);
            cz[r][a] = DIM == 3 ? tb2->pc[fi[2]][a] : 0;
            wz[r][a] = DIM == 3 ? T(tb2->pw[fi[2]][a]) : T(a == 0 ? 1 : 0);
            const bool okx = cx[r][a] >= 0 && cx[r][a] < cb.m[0];
            const bool oky = cy[r][a] >= 0 && cy[r][a] < cb.m[1];
            const bool okz = DIM == 2 || (cz[r][a] >= 0 && cz[r][a] < cb.m[2]);
            wx[r][a] = okx ? wx[r][a] : T(0);
            cx[r][a] = okx ? cx[r][a] : 0;
            wy[r][a] = oky ? wy[r][a] : T(0);
            cy[r][a] = oky ? cy[r][a] : 0;
            wz[r][a] = okz ? wz[r][a] : T(0);
            cz[r][a] = okz ? cz[r][a] : 0;
          }
        }
#pragma unroll
        for (int r = 0; r < PB; ++r) {
          T acc = T(0);
#pragma unroll
          for (int c = 0; c < (DIM == 3 ? 2 : 1); ++c)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
              for (int a = 0; a < 2; ++a)
                acc += wx[r][a] * wy[r][b] * wz[r][c] * Xc[cx[r][a] + cb.m[0] * (cy[r][b] + cb.m[1] * cz[r][c])];
          if (i0 + 64 * r < fb.n) Xk[i0 + 64 * r] += acc;
          wf[r].step();
        }
      }
      wave_sync();
    }
    if (k == 0 && !WARM)
      residual<DIM, T, ST, true>(Rk, Bk, Xk, fb, stn[k], pa.lng[k], r, md);
    else
      residual<DIM, T, ST, false>(Rk, Bk, Xk, fb, stn[k], pa.lng[k], r, md);
    slot_table<DIM>(tab, fb.m[0], fb.m[1]);
    sweep<T, true>(Rk, bf, tab);
    sweep<T, false>(Rk, bb, tab);
    for (int i = threadIdx.x; i < fb.n; i += 64) Xk[i] += Rk[i];
    wave_sync();
  }
  // scatter-add the correction, or (dense mode, training data of the patch
  // network) write it divided by the patch's scale into the patch's
  // (2p-1)^d grid: grid point g_d = level-0 node - (v_d p - p + 1)
  {
    const T *X0 = lds_vec<DIM, T, WARM>(lds, pa, v, 0, 0);
    if (dense) {
      const double inv = 1.0 / dscale[j];
      Walk<DIM> w(b0, threadIdx.x, 64);
      for (int i = threadIdx.x; i < b0.n; i += 64, w.step())
        dense[int64_t(j) * G3 + grid_q(w)] = float(double(X0[i]) * inv);
    } else {
      Walk<DIM> w(b0, threadIdx.x, 64);
      if (WARM) {
        const double sc = dscale[blockIdx.x];
        const float *yj = wy + int64_t(blockIdx.x) * G3;
        for (int i = threadIdx.x; i < b0.n; i += 64, w.step()) {
          const double c = double(X0[i]) + double(yj[grid_q(w)]) * sc;
          unsafeAtomicAdd(z + walk_uidx<DIM>(b0, w, md), pa.pou ? c * pou_weight<DIM>(b0, w, md.p) : c);
        }
      } else {
        for (int i = threadIdx.x; i < b0.n; i += 64, w.step()) {
          const double c = double(X0[i]);
          const double v = pa.pou ? c * pou_weight<DIM>(b0, w, md.p) : c;
          double *zu = z + walk_uidx<DIM>(b0, w, md);
          if (pa.plain)
            *zu += v;
          else
            unsafeAtomicAdd(zu, v);
        }
      }
    }
  }
}

// gfx950: 160 KB of LDS per CU, all of it addressable by one workgroup.
constexpr int kMaxDynLds = 160 * 1024;

template <int DIM, typename T, typename ST, bool WARM>
hipError_t prepare_t() {
  constexpr int W = DIM == 3 ? 26 : 8;
  hipError_t e = hipFuncSetAttribute((const void *)k_patch_vcycle<DIM, T, ST, W, WARM>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, kMaxDynLds);
  if (e != hipSuccess || WARM) return e;
  return hipFuncSetAttribute((const void *)k_patch_vcycle<DIM, T, ST, W, false, true>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, kMaxDynLds);
}

static_assert(sizeof(PatchJobs) <= 4000, "the jobs travel as a kernel argument (4 KiB at most)");

template <int DIM, typename T, typename ST>
hipError_t launch_jobs_t(const PatchJobs &pj, int64_t blocks, hipStream_t st) {
  constexpr int W = DIM == 3 ? 26 : 8;
  size_t lds = 0;
  for (int k = 0; k < pj.njobs; ++k)
    lds = std::max(lds, lds_values<DIM, false>(pj.p[k]) * sizeof(T) + kSlotTableBytes);
  if (lds > size_t(kMaxDynLds) || blocks > int64_t(INT32_MAX)) return hipErrorInvalidValue;
  if (blocks <= 0) return hipSuccess;
  k_patch_vcycle<DIM, T, ST, W, false, true><<<int(blocks), 64, lds, st>>>(pj, nullptr, nullptr, nullptr, nullptr,
                                                                         nullptr, nullptr, 0);
  return hipGetLastError();
}

template <int DIM, typename T, typename ST, bool WARM>
hipError_t launch_t(const PatchArgs &pa, int npatch, const double *r, double *z, const double *flag,
                    float *dense, const double *dscale, const float *wy, int jfirst, hipStream_t st) {
  constexpr int W = DIM == 3 ? 26 : 8;
  const size_t lds = lds_values<DIM, WARM>(pa) * sizeof(T) + kSlotTableBytes;
  if (lds > size_t(kMaxDynLds)) return hipErrorInvalidValue;
  if (npatch <= 0) return hipSuccess;
  k_patch_vcycle<DIM, T, ST, W, WARM><<<npatch, 64, lds, st>>>(pa, r, z, flag, dense, dscale, wy, jfirst);
  return hipGetLastError();
}

}  // namespace

hipError_t prepare_patch_vcycle(const PatchArgs &pa) {
  if (pa.md.dim == 3) {
    hipError_t e = pa.fp32 ? prepare_t<3, float, float, false>() : prepare_t<3, double, double, false>();
    if (e != hipSuccess) return e;
    return pa.fp32 ? prepare_t<3, float, float, true>() : prepare_t<3, double, double, true>();
  }
  return pa.fp32 ? prepare_t<2, float, float, false>() : prepare_t<2, double, double, false>();
}

hipError_t launch_patch_vcycle(const PatchArgs &pa, int npatch, const double *r, double *z,
                               const double *flag, hipStream_t st, float *dense,
                               const double *dscale) {
  if (pa.plain && !dense) {
    // one launch per vertex-parity class, in class order
    const int nclass = pa.md.dim == 3 ? 8 : 4;
    for (int color = 0; color < nclass; ++color) {
      PatchArgs pc = pa;
      pc.plain = 0;
      pc.color = color;
      pc.perm = nullptr;
      pc.nrhs = 0;
      int cnt = 1;
      for (int d = 0; d < pa.md.dim; ++d) cnt *= (pa.nv[d] - ((color >> d) & 1) + 1) / 2;
      pc.plain = 1;
      hipError_t e;
      if (pa.fp32)
        e = pa.md.dim == 3 ? launch_t<3, float, float, false>(pc, cnt, r, z, flag, nullptr, nullptr, nullptr, 0, st)
                           : launch_t<2, float, float, false>(pc, cnt, r, z, flag, nullptr, nullptr, nullptr, 0, st);
      else
        e = pa.md.dim == 3 ? launch_t<3, double, double, false>(pc, cnt, r, z, flag, nullptr, nullptr, nullptr, 0, st)
                           : launch_t<2, double, double, false>(pc, cnt, r, z, flag, nullptr, nullptr, nullptr, 0, st);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  if (pa.fp32) {
    if (pa.md.dim == 3)
      return launch_t<3, float, float, false>(pa, npatch, r, z, flag, dense, dscale, nullptr, 0, st);
    return launch_t<2, float, float, false>(pa, npatch, r, z, flag, dense, dscale, nullptr, 0, st);
  }
  if (pa.md.dim == 3)
    return launch_t<3, double, double, false>(pa, npatch, r, z, flag, dense, dscale, nullptr, 0, st);
  return launch_t<2, double, double, false>(pa, npatch, r, z, flag, dense, dscale, nullptr, 0, st);
}

hipError_t launch_patch_vcycle_multi(const PatchArgs &pa, int npatch, int nrhs,
                                     const double *const *r, double *const *z,
                                     const double *const *flags, hipStream_t st) {
  if (nrhs < 1 || nrhs > kMaxRhs || pa.plain || !r || !z) return hipErrorInvalidValue;
  int J = 1;
  for (int d = 0; d < pa.md.dim; ++d) J *= pa.nv[d];
  if (npatch != J) return hipErrorInvalidValue;
  if (npatch <= 0) return hipSuccess;
  PatchArgs pm = pa;
  pm.nrhs = nrhs;
  for (int k = 0; k < kMaxRhs; ++k) {
    pm.rs[k] = k < nrhs ? r[k] : nullptr;
    pm.zs[k] = k < nrhs ? z[k] : nullptr;
    pm.flags[k] = k < nrhs && flags ? flags[k] : nullptr;
    if (k < nrhs && (!pm.rs[k] || !pm.zs[k])) return hipErrorInvalidValue;
  }
  const int64_t blocks = int64_t((npatch + 7) / 8) * 8 * nrhs;
  if (blocks > int64_t(INT32_MAX)) return hipErrorInvalidValue;
  if (pa.fp32) {
    if (pa.md.dim == 3)
      return launch_t<3, float, float, false>(pm, int(blocks), nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0, st);
    return launch_t<2, float, float, false>(pm, int(blocks), nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0, st);
  }
  if (pa.md.dim == 3)
    return launch_t<3, double, double, false>(pm, int(blocks), nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0, st);
  return launch_t<2, double, double, false>(pm, int(blocks), nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0, st);
}

hipError_t launch_patch_vcycle_jobs(const PatchArgs *jobs, int njobs, hipStream_t st) {
  if (!jobs || njobs < 1 || njobs > kMaxJobs) return hipErrorInvalidValue;
  PatchJobs pj{};
  pj.njobs = njobs;
  int64_t blocks = 0;
  for (int k = 0; k < njobs; ++k) {
    const PatchArgs &a = jobs[k];
    if (a.md.dim != jobs[0].md.dim || a.fp32 != jobs[0].fp32 || a.plain || a.color >= 0 ||
        a.nrhs < 1 || a.nrhs > kMaxRhs)
      return hipErrorInvalidValue;
    for (int i = 0; i < a.nrhs; ++i)
      if (!a.rs[i] || !a.zs[i]) return hipErrorInvalidValue;
    int64_t J = 1;
    for (int d = 0; d < a.md.dim; ++d) J *= a.nv[d];
    pj.p[k] = a;
    pj.block0[k] = int(std::min<int64_t>(blocks, INT32_MAX));
    blocks += (J + 7) / 8 * 8 * a.nrhs;
  }
  if (blocks > int64_t(INT32_MAX)) return hipErrorInvalidValue;
  pj.block0[njobs] = int(blocks);
  if (jobs[0].fp32)
    return jobs[0].md.dim == 3 ? launch_jobs_t<3, float, float>(pj, blocks, st)
                               : launch_jobs_t<2, float, float>(pj, blocks, st);
  return jobs[0].md.dim == 3 ? launch_jobs_t<3, double, double>(pj, blocks, st)
                             : launch_jobs_t<2, double, double>(pj, blocks, st);
}

hipError_t launch_patch_vcycle_warm(const PatchArgs &pa, int first, int count, const double *r,
                                    double *z, const float *y, const double *scale,
                                    const double *flag, hipStream_t st) {
  if (pa.md.dim != 3 || !y || !scale || first < 0 || count < 0 || pa.plain) return hipErrorInvalidValue;
  PatchArgs pw = pa;
  pw.perm = nullptr;  // predictions and scales are indexed by block
  pw.nrhs = 0;
  if (pa.fp32)
    return launch_t<3, float, float, true>(pw, count, r, z, flag, nullptr, scale, y, first, st);
  return launch_t<3, double, double, true>(pw, count, r, z, flag, nullptr, scale, y, first, st);
}

}  // namespace lor
