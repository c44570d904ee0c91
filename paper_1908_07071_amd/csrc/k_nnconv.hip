// Fused 3x3x3 convolution layer of the patch network (inference and
// training forward), as an implicit GEMM on BF16 MFMA: no im2col matrix is
// formed.  One workgroup (four wavefronts) per patch at a time; the patch's
// activation planes z-1, z, z+1 sit in LDS with a zero halo (so the zero
// padding of the convolution costs nothing) and a fixed row pitch, the next
// plane is loaded while the current one is computed.  Each wavefront keeps the weights of its
// 16-wide output-channel tile in registers for the whole kernel and computes
// 16-point M-tiles of a plane: per K-step of 16 (one kernel offset and 16
// input channels) one 8-byte LDS read and one v_mfma_f32_16x16x16bf16.
//
// Layouts (as the explicit path): activations [n G^3 + q][Cin] bf16, q = gx
// + G (gy + G gz); weights [Kp][Np] bf16 with row k Cin + c, k = (dx+1) +
// 3 (dy+1) + 9 (dz+1); bias [Np]; pre-activations [row][Np] float.
#include <hip/hip_runtime.h>

#include "lor_internal.h"

namespace lor {

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ inline uint16_t f2bf_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return uint16_t((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}

constexpr int pad16c(int x) { return (x + 15) & ~15; }
// LDS row pitch of one grid point (bf16 values): padded against bank
// conflicts, a multiple of 4 so 8-byte reads stay aligned
constexpr int cpad(int cin) { return cin == 2 ? 2 : cin + 8; }
constexpr int kSlots = 4;  // plane slots: three in use, one loading
constexpr int kRP = 17;    // LDS row pitch of a plane in points (G + 2 <= 17): every
                           // neighbour offset is then a compile-time immediate

// LDS values (uint16) of one workgroup: kSlots planes and two output
// staging buffers (bf16 [G^2][COUT], or float [G^2] for the output layer)
__host__ __device__ constexpr int conv_plane(int G, int cin) { return (G + 2) * kRP * cpad(cin); }
__host__ __device__ constexpr int conv_stage(int G, int cout, bool last) {
  return last ? 2 * G * G : G * G * cout;
}

// CIN input channels, NT output tiles of 16 channels, COUT output channels,
// LAST: the output layer (masked, one channel).  Each wavefront computes
// every output tile of its M-tiles (m = wave, wave + 4, ...), so an A
// fragment read from LDS serves NT MFMAs.
template <int CIN, int NT, int COUT, bool LAST>
__global__ __launch_bounds__(256) void k_conv3(const uint16_t *__restrict__ ain, int nb, int G,
                                               const uint16_t *__restrict__ Wf,
                                               const float *__restrict__ bias,
                                               float *__restrict__ zout, uint16_t *__restrict__ aout,
                                               const float *__restrict__ X, float *__restrict__ y,
                                               const double *flag) {
  if (flag && flag[S_DONE] != 0.0) return;  // uniform over the grid
  constexpr int KP = pad16c(27 * CIN), KS = KP / 16, NP = NT * 16, CP = cpad(CIN);
  constexpr int UM = 2;       // M-tiles in flight per wavefront (UM NT MFMA chains)
  constexpr int kGroup = 3;   // K-steps between scheduling barriers
  extern __shared__ __align__(16) uint16_t pl[];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int G2 = G * G, G3 = G2 * G, PP = conv_plane(G, CIN);
  const int OS = conv_stage(G, COUT, LAST);
  uint16_t *stage0 = pl + kSlots * PP;  // two staging buffers of OS values
  const int MT = (G2 + 15) / 16;
  // the weights of every output tile in fragment order (B[4(l/16)+t][l%16]
  // of K-step s and tile nt at ((s NT + nt) 64 + l) 4 + t)
  bf16x4 w[NT][KS];
#pragma unroll
  for (int s = 0; s < KS; ++s)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
      w[nt][s] = *reinterpret_cast<const bf16x4 *>(Wf + ((s * NT + nt) * 64 + lane) * 4);
  float bv[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) bv[nt] = bias[nt * 16 + (lane & 15)];
  for (int i = threadIdx.x; i < kSlots * PP; i += 256) pl[i] = 0;  // halos stay zero
  __syncthreads();
  // one plane of a patch into a slot (interior points only); out-of-grid
  // planes are zero
  constexpr int VEC = CIN == 2 ? 2 : 4;  // values per item
  constexpr int IPP = CIN / VEC;         // items per point
  const int items = G2 * IPP;
  constexpr int RI = (15 * 15 * IPP + 255) / 256;  // items per thread held in registers (G <= 15)
  typedef uint32_t word2 __attribute__((ext_vector_type(2)));
  auto fetch = [&](int n, int gz, word2 (&buf)[RI]) {
#pragma unroll
    for (int r = 0; r < RI; ++r) {
      const int it = threadIdx.x + 256 * r;
      buf[r] = word2{0u, 0u};
      if (it < items && gz >= 0 && gz < G) {
        const int pt = it / IPP, cq = it % IPP;
        const uint16_t *src = ain + (int64_t(n) * G3 + int64_t(gz) * G2 + pt) * CIN + cq * VEC;
        if (VEC == 4)
          buf[r] = *reinterpret_cast<const word2 *>(src);
        else
          buf[r].x = *reinterpret_cast<const uint32_t *>(src);
      }
    }
  };
  auto store = [&](int slot, const word2 (&buf)[RI]) {
    uint16_t *dst = pl + slot * PP;
#pragma unroll
    for (int r = 0; r < RI; ++r) {
      const int it = threadIdx.x + 256 * r;
      if (it < items) {
        const int pt = it / IPP, cq = it % IPP;
        const int px = pt % G, py = pt / G;
        uint16_t *d = dst + ((py + 1) * kRP + px + 1) * CP + cq * VEC;
        if (VEC == 4)
          *reinterpret_cast<word2 *>(d) = buf[r];
        else
          *reinterpret_cast<uint32_t *>(d) = buf[r].x;
      }
    }
  };
  // a staged output plane to global memory: contiguous rows, 16-byte stores
  // (ReLU bf16 activations) or the masked float output
  auto flush = [&](int n, int z, const uint16_t *st) {
    const int64_t row0 = int64_t(n) * G3 + int64_t(z) * G2;
    if (LAST) {
      const float *sf = reinterpret_cast<const float *>(st);
      for (int i = threadIdx.x; i < G2; i += 256) y[row0 + i] = sf[i] * X[(row0 + i) * 2 + 1];
    } else {
      constexpr int PER = 8;  // bf16 per 16-byte store
      const int nv = G2 * COUT / PER;
      uint4 *dst = reinterpret_cast<uint4 *>(aout + row0 * COUT);
      const uint4 *src = reinterpret_cast<const uint4 *>(st);
      for (int i = threadIdx.x; i < nv; i += 256) dst[i] = src[i];
    }
  };
  for (int n = blockIdx.x; n < nb; n += gridDim.x) {
    word2 buf[RI];
    // planes -1, 0, 1 into slots 0, 1, 2 (slot of plane gz: (gz + 1) mod 4)
    for (int gz = -1; gz <= 1; ++gz) {
      fetch(n, gz, buf);
      store(gz + 1, buf);
    }
    __syncthreads();
    for (int z = 0; z < G; ++z) {
      if (z > 0) flush(n, z - 1, stage0 + ((z - 1) & 1) * OS);
      fetch(n, z + 2, buf);  // in flight during the plane's MFMAs
      uint16_t *st = stage0 + (z & 1) * OS;
      // slot offsets of planes z-1, z, z+1 as element indices into pl (kept
      // as integers, so that every access stays an LDS access)
      const int sl[3] = {((z) % kSlots) * PP, ((z + 1) % kSlots) * PP, ((z + 2) % kSlots) * PP};
      for (int m = wv; m < MT; m += UM * 4) {
        int mm[UM];
        int bz[UM][3];  // per tile and plane: LDS index of the (-1, -1) neighbour + channel group
#pragma unroll
        for (int u = 0; u < UM; ++u) {
          mm[u] = m + u * 4 < MT ? m + u * 4 : m;
          const int pv = min(mm[u] * 16 + (lane & 15), G2 - 1);
          const int corner = ((pv / G) * kRP + pv % G) * CP + (CIN % 16 == 0 ? 4 * (lane >> 4) : 0);
#pragma unroll
          for (int d = 0; d < 3; ++d) bz[u][d] = sl[d] + corner;
        }
        f32x4 acc[UM][NT];
#pragma unroll
        for (int u = 0; u < UM; ++u)
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) acc[u][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < KS; ++s) {
#pragma unroll
          for (int u = 0; u < UM; ++u) {
            bf16x4 a;
            if (CIN % 16 == 0) {
              const int k = (s * 16) / CIN, c0 = (s * 16) % CIN;
              const int dx = k % 3 - 1, dy = (k / 3) % 3 - 1, dz = k / 9;
              a = *reinterpret_cast<const bf16x4 *>(&pl[bz[u][dz] + ((dy + 1) * kRP + dx + 1) * CP + c0]);
            } else {
              // CIN = 2: K index j = k * 2 + c; columns past 27 * 2 are zero
#pragma unroll
              for (int t = 0; t < 4; ++t) {
                const int jj = s * 16 + 4 * (lane >> 4) + t;
                const int k = min(jj >> 1, 26), c = jj & 1;
                const int dx = k % 3 - 1, dy = (k / 3) % 3 - 1, dz = k / 9;
                const int sb = dz == 0 ? bz[u][0] : (dz == 1 ? bz[u][1] : bz[u][2]);
                const short v = short(pl[sb + ((dy + 1) * kRP + dx + 1) * CP + c]);
                a[t] = jj < 54 ? v : short(0);
              }
            }
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
              acc[u][nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, w[nt][s], acc[u][nt], 0, 0, 0);
          }
          // bounds how far the scheduler hoists the LDS reads (register use)
          if (s % kGroup == kGroup - 1) __builtin_amdgcn_sched_barrier(0);
        }
        // C[4(l/16)+t][l%16]: points mm*16 + 4(l/16) + t, channel nt*16 + l%16,
        // staged in LDS (pre-activations straight to zout when kept)
#pragma unroll
        for (int u = 0; u < UM; ++u) {
          if (u > 0 && mm[u] == m) break;  // tiles past the plane repeat tile m
#pragma unroll
          for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
              const int pr = mm[u] * 16 + 4 * (lane >> 4) + t;
              const int o = nt * 16 + (lane & 15);
              if (pr < G2) {
                const float v = acc[u][nt][t] + bv[nt];
                if (zout) zout[(int64_t(n) * G3 + int64_t(z) * G2 + pr) * NP + o] = v;
                if (LAST) {
                  if (o == 0) reinterpret_cast<float *>(st)[pr] = v;
                } else if (o < COUT) {
                  st[pr * COUT + o] = f2bf_rne(v > 0.f ? v : 0.f);
                }
              }
            }
        }
      }
      store((z + 3) % kSlots, buf);  // plane z + 2: its slot held plane z - 2
      __syncthreads();
    }
    flush(n, G - 1, stage0 + ((G - 1) & 1) * OS);
    __syncthreads();  // the staging buffers are reused by the next patch
  }
}

// Wf[((s NT + nt) 64 + l) 4 + t] = Wb[(16 s + 4 (l / 16) + t) Np + 16 nt + l % 16]
__global__ void k_frag(const uint16_t *__restrict__ Wb, int Kp, int Np, uint16_t *__restrict__ Wf) {
  const int NT = Np / 16;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < int64_t(Kp) * Np;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int t = int(i % 4), l = int((i / 4) % 64);
    const int sn = int(i / 256), nt = sn % NT, s = sn / NT;
    Wf[i] = Wb[int64_t(16 * s + 4 * (l / 16) + t) * Np + 16 * nt + l % 16];
  }
}

template <int CIN, int NT, int COUT, bool LAST>
hipError_t launch_conv(const uint16_t *ain, int nb, int G, const uint16_t *Wf, const float *bias,
                       float *zout, uint16_t *aout, const float *X, float *y, const double *flag,
                       hipStream_t st) {
  const size_t lds = (size_t(kSlots) * conv_plane(G, CIN) + 2 * size_t(conv_stage(G, COUT, LAST))) *
                     sizeof(uint16_t);
  const int grid = nb < 2048 ? nb : 2048;
  k_conv3<CIN, NT, COUT, LAST><<<grid, 256, lds, st>>>(ain, nb, G, Wf, bias, zout, aout, X, y, flag);
  return hipGetLastError();
}

}  // namespace

bool nn_conv_supported(int channels, int G) {
  return (channels == 16 || channels == 32) && G >= 3 && G <= 15;
}

hipError_t nn_conv_prepare(int channels) {
  // the LDS limit of every instantiation, set once when a network is created
  hipError_t e = hipSuccess;
  auto set = [&](const void *f) {
    if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  };
  if (channels == 16) {
    set((const void *)k_conv3<2, 1, 16, false>);
    set((const void *)k_conv3<16, 1, 16, false>);
    set((const void *)k_conv3<16, 1, 1, true>);
  } else if (channels == 32) {
    set((const void *)k_conv3<2, 2, 32, false>);
    set((const void *)k_conv3<32, 2, 32, false>);
    set((const void *)k_conv3<32, 1, 1, true>);
  } else {
    return hipErrorInvalidValue;
  }
  return e;
}

hipError_t nn_conv_frag(const uint16_t *Wb, int Kp, int Np, uint16_t *Wf, hipStream_t st) {
  if (Kp % 16 || Np % 16 || Kp <= 0 || Np <= 0) return hipErrorInvalidValue;
  const int64_t n = int64_t(Kp) * Np;
  k_frag<<<int((n + 255) / 256), 256, 0, st>>>(Wb, Kp, Np, Wf);
  return hipGetLastError();
}

hipError_t nn_conv_layer(int channels, int layer, const uint16_t *ain, int nb, int G,
                         const uint16_t *Wf, const float *bias, float *zout, uint16_t *aout,
                         const float *X, float *y, const double *flag, hipStream_t st) {
  if (!nn_conv_supported(channels, G) || nb <= 0) return hipErrorInvalidValue;
  if (channels == 16) {
    if (layer == 0) return launch_conv<2, 1, 16, false>(ain, nb, G, Wf, bias, zout, aout, X, y, flag, st);
    if (layer == 1) return launch_conv<16, 1, 16, false>(ain, nb, G, Wf, bias, zout, aout, X, y, flag, st);
    return launch_conv<16, 1, 1, true>(ain, nb, G, Wf, bias, zout, aout, X, y, flag, st);
  }
  if (layer == 0) return launch_conv<2, 2, 32, false>(ain, nb, G, Wf, bias, zout, aout, X, y, flag, st);
  if (layer == 1) return launch_conv<32, 2, 32, false>(ain, nb, G, Wf, bias, zout, aout, X, y, flag, st);
  return launch_conv<32, 1, 1, true>(ain, nb, G, Wf, bias, zout, aout, X, y, flag, st);
}

}  // namespace lor
