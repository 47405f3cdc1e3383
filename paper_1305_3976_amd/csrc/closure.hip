// closure.hip -- the learned-closure kernels of libibgm.so (C ABI in
// include/ibgm_closure.h): 3x3x3 convolutions on the gfx950 matrix cores
// (v_mfma_f32_32x32x16_bf16: BF16 operands, FP32 accumulation), their two
// gradients, the loss, Adam, and the MAC restriction / gather / apply steps
// that connect the network to the IB-GM fields.
//
// Convolution as an implicit GEMM.  For one output row of 32 voxels along x
// and one tap, the product [32 output channels x 16 input channels] x [16 x
// 32 voxels] (the transposed form, so that a lane's accumulators are
// consecutive channels of one voxel) is one matrix-core instruction; 27 taps
// x (ci/16) of them build the 32 x 32 output block.  A workgroup (4 waves)
// keeps every packed weight fragment of the layer in LDS for its whole life
// and walks output tiles of 32 x 4 x 4 voxels: it stages the tile's input
// halo (34 x 6 x 6 voxels, all channels) in LDS, and each wave accumulates
// the four rows of one z-slice.
// Matrix-core lane layout (32x32x16): lane l supplies A[row l%32][k
// 8(l/32)..+7] and B[k 8(l/32)..+7][col l%32]; accumulator j of lane l is
// D[8(j/4) + 4(l/32) + j%4][l%32].
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <type_traits>

#include "errors.h"
#include "ibgm_closure.h"

namespace {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int TX = 32, TY = 4, TZ = 4;               // output tile (voxels); TZ = waves
constexpr int HX = TX + 2, HY = TY + 2, HZ = TZ + 2;  // its input halo
constexpr int NT = 256;                               // threads per workgroup
constexpr int CO = 32;                                // output channels
constexpr int WG_CONV = 256;                          // persistent workgroups (1 per CU)

__device__ __forceinline__ int wrapi(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

// Periodic index for -n <= i < 2n (one compare-and-add instead of a modulo).
__device__ __forceinline__ int wrap1(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

struct ConvArgs {
  const bf16 *x;      // [B][D2][D1][D0][CI]
  const bf16 *wp;     // packed fragments [27][CI/16][64][8]
  const float *bias;  // [32] or null
  const bf16 *mask;   // [B][E2][E1][E0][32] or null: output *= (mask > 0)
  void *y;            // [B][E2][E1][E0][ystride]
  int B, D0, D1, D2, E0, E1, E2;
  int off, wrap;  // wrap: 0 = zeros outside, 1 = periodic (dims >= TX + 2), 2 = periodic
  int relu, out_f32, co_store, ystride;
  int nt0, nt1, nt2, ntiles;
  int qoff_ok;      // a halo's extent, HZ D1 D0 voxels, spans < 2^31 bytes
  float *add[3];    // k_conv_n16<.., true>: add[c][voxel] += add_scale * output c (c < 3)
  float add_scale;
};

// Stage the input halo of the tile at (b, ox0, oy0, oz0) in LDS: voxel v of
// the halo (x fastest) at byte v * VS, CI channels, zeros outside the input
// unless the indices wrap.
template <int CI, int VS>
__device__ __forceinline__ void load_halo(unsigned char *sh, const bf16 *x, int b, int ox0,
                                          int oy0, int oz0, int D0, int D1, int D2, int off,
                                          int wrap) {
  constexpr int CH = CI / 8;  // 16-byte chunks per voxel
  for (int c = threadIdx.x; c < HX * HY * HZ * CH; c += NT) {
    const int v = c / CH, part = c - v * CH;
    const int hx = v % HX, hy = (v / HX) % HY, hz = v / (HX * HY);
    int gx = ox0 + hx + off, gy = oy0 + hy + off, gz = oz0 + hz + off;
    uint4 val = make_uint4(0, 0, 0, 0);
    bool in = true;
    if (wrap) {
      gx = wrapi(gx, D0), gy = wrapi(gy, D1), gz = wrapi(gz, D2);
    } else {
      in = gx >= 0 && gx < D0 && gy >= 0 && gy < D1 && gz >= 0 && gz < D2;
    }
    if (in) {
      const size_t vox = (((size_t)b * D2 + gz) * D1 + gy) * D0 + gx;
      val = *reinterpret_cast<const uint4 *>(x + vox * CI + part * 8);
    }
    *reinterpret_cast<uint4 *>(sh + v * VS + part * 16) = val;
  }
}

struct TileXYZ {
  int b, ox0, oy0, oz0;
};

__device__ __forceinline__ TileXYZ tile_xyz(int tile, int nt0, int nt1, int nt2) {
  int r = tile;
  const int t0 = r % nt0;
  r /= nt0;
  const int t1 = r % nt1;
  r /= nt1;
  const int t2 = r % nt2;
  return {r / nt2, t0 * TX, t1 * TY, t2 * TZ};
}

// Halo chunk metadata of one thread, fixed for the kernel's life: chunk c of
// a tile's input halo (16 bytes of one voxel's channels) lies at halo voxel
// (hx, hy, hz), 16-byte part `part` of the voxel, and goes to LDS byte
// v VS + 16 part (SWZ, two parts per voxel: the parts of voxels with bit 2
// of v set trade places, so that lanes reading the same part of voxels v and
// v + 4 meet different LDS banks).  Packed as hx | hy << 6 | hz << 9 |
// part << 12 | (LDS byte / 16) << 14 (27 bits); -1 for chunk numbers past
// the halo.
template <int CI, int VS, bool SWZ = false>
__device__ __forceinline__ int halo_meta(int c) {
  constexpr int CH = CI / 8;
  if (c >= HX * HY * HZ * CH) return -1;
  const int v = c / CH, part = c - v * CH;
  const int hx = v % HX, hy = (v / HX) % HY, hz = v / (HX * HY);
  const int slot = SWZ ? part ^ ((v >> 2) & 1) : part;
  return hx | hy << 6 | hz << 9 | part << 12 | ((v * VS + slot * 16) >> 4) << 14;
}

// Load one halo chunk of the tile whose halo starts at input voxel (gx0, gy0,
// gz0) of batch item b.  WRAP: 0 = zeros outside the input, 1 = periodic with
// every dimension >= the halo (one compare-and-add), 2 = periodic, any size.
template <int CI, int WRAP>
__device__ __forceinline__ uint4 halo_load(const ConvArgs &a, int meta, int b, int gx0, int gy0,
                                           int gz0) {
  uint4 val = make_uint4(0, 0, 0, 0);
  if (meta < 0) return val;
  int gx = gx0 + (meta & 63), gy = gy0 + ((meta >> 6) & 7), gz = gz0 + ((meta >> 9) & 7);
  if (WRAP == 1) {
    gx = wrap1(gx, a.D0), gy = wrap1(gy, a.D1), gz = wrap1(gz, a.D2);
  } else if (WRAP == 2) {
    gx = wrapi(gx, a.D0), gy = wrapi(gy, a.D1), gz = wrapi(gz, a.D2);
  } else if (gx < 0 || gx >= a.D0 || gy < 0 || gy >= a.D1 || gz < 0 || gz >= a.D2) {
    return val;
  }
  const int64_t vox = (((int64_t)b * a.D2 + gz) * a.D1 + gy) * a.D0 + gx;
  return *reinterpret_cast<const uint4 *>(a.x + vox * CI + ((meta >> 12) & 3) * 8);
}

// Byte offset of a thread's halo chunk from the halo's first voxel when the
// halo lies inside the input (no wrap): fixed for the kernel, since it
// depends only on the chunk and the input's row and plane sizes.
template <int CI>
__device__ __forceinline__ uint32_t halo_qoff(int meta, int D0, int D1) {
  if (meta < 0) return 0u;
  const int hx = meta & 63, hy = (meta >> 6) & 7, hz = (meta >> 9) & 7, part = (meta >> 12) & 3;
  return (uint32_t)(((hz * D1 + hy) * D0 + hx) * (CI * 2) + part * 16);
}

// Fetch a tile's halo chunks into registers, every load issued before any
// is used.  A tile whose halo lies inside the input reads chunk q at the
// halo's base address plus qoff[q] (one add per load); the tiles at the
// input's faces take halo_load's wrap or zero-fill arithmetic.
template <int CI, int WRAP, int PER>
__device__ __forceinline__ void fetch_halo(const ConvArgs &a, const int (&meta)[PER],
                                           const uint32_t (&qoff)[PER], const TileXYZ &t,
                                           uint4 (&pre)[PER]) {
  constexpr int NCHUNK = HX * HY * HZ * (CI / 8);
  const int gx0 = t.ox0 + a.off, gy0 = t.oy0 + a.off, gz0 = t.oz0 + a.off;
  const bool inside = a.qoff_ok && gx0 >= 0 && gx0 + HX <= a.D0 && gy0 >= 0 &&
                      gy0 + HY <= a.D1 && gz0 >= 0 && gz0 + HZ <= a.D2;
  if (inside) {
    const char *base = reinterpret_cast<const char *>(a.x) +
                       ((((int64_t)t.b * a.D2 + gz0) * a.D1 + gy0) * a.D0 + gx0) * (CI * 2);
#pragma unroll
    for (int q = 0; q < PER; q++) {
      pre[q] = make_uint4(0, 0, 0, 0);
      if ((q + 1) * NT <= NCHUNK || meta[q] >= 0)
        pre[q] = *reinterpret_cast<const uint4 *>(base + qoff[q]);
    }
  } else {
#pragma unroll
    for (int q = 0; q < PER; q++) pre[q] = halo_load<CI, WRAP>(a, meta[q], t.b, gx0, gy0, gz0);
  }
}

// Output channel held in row r of the transposed 32 x 32 product: rows are
// permuted so that the 16 accumulators of a lane are 16 consecutive channels
// (lane l, accumulator j: row 8 (j/4) + 4 (l/32) + j%4, channel 16 (l/32) + j).
__device__ __forceinline__ int row_channel(int r) { return 16 * ((r >> 2) & 1) + 4 * (r >> 3) + (r & 3); }

// Copy the packed weight fragments into LDS as matrix-core A operands: lane l
// of fragment f takes packed lane 32 (l/32) + row_channel(l%32) (PERM), or
// lane l itself.  Eight loads of a thread are in flight before their stores.
template <int N, bool PERM>
__device__ __forceinline__ void copy_weights(unsigned char *sw, const bf16 *wp) {
  constexpr int PERW = (N + NT - 1) / NT, BATCH = 8;
#pragma unroll
  for (int q0 = 0; q0 < PERW; q0 += BATCH) {
    uint4 w[BATCH];
#pragma unroll
    for (int q = 0; q < BATCH; q++) {
      const int c = threadIdx.x + (q0 + q) * NT;
      int src = c;
      if (PERM) src = (c & ~31) | row_channel(c & 31);
      w[q] = (q0 + q < PERW && c < N) ? reinterpret_cast<const uint4 *>(wp)[src]
                                      : make_uint4(0, 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < BATCH; q++) {
      const int c = threadIdx.x + (q0 + q) * NT;
      if (q0 + q < PERW && c < N) reinterpret_cast<uint4 *>(sw)[c] = w[q];
    }
  }
}

// Forward convolution (and, with adjoint packing, the input gradient).
// Wave w computes the 4 output rows (y = 0..3) of z-slice w of the tile as
// the transposed product Y^T = W^T X^T: the weights are the A operand and the
// halo row the B operand, so each lane ends with 16 consecutive output
// channels of one voxel and stores them as two 16-byte writes (VEC), or
// channel by channel (any co_store, y_stride, FP32 output).  For each (tz,
// tx) a wave keeps the three weight fragments of ty = 0..2 in registers and
// walks the 6 halo rows once: a halo row hy feeds output rows hy - ty, so
// each B fragment read from LDS serves up to three matrix-core products.  A
// tile's halo is fetched with all of a thread's loads in flight before any is
// stored to LDS, from per-thread chunk coordinates computed once.  With 16
// input channels the halo is stored unpadded (32-byte voxels, the two halves
// swizzled against bank conflicts) so that weights and halo fit twice in one
// CU's LDS: two workgroups per CU, one's halo fetch beside the other's
// products.
template <int CI, int WRAP, bool VEC>
__global__ __launch_bounds__(NT, CI == 16 ? 2 : 1) void k_conv(ConvArgs a) {
  constexpr int KS = CI / 16;
  constexpr bool SWZ = CI == 16;
  constexpr int VS = SWZ ? CI * 2 : CI * 2 + 16;  // voxel stride in LDS (bytes)
  constexpr int NCHUNK = HX * HY * HZ * (CI / 8);
  constexpr int PER = (NCHUNK + NT - 1) / NT;
  __shared__ __align__(16) unsigned char sw[27 * KS * 64 * 16];
  __shared__ __align__(16) unsigned char sh[HX * HY * HZ * VS];
  copy_weights<27 * KS * 64, true>(sw, a.wp);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 31, grp = lane >> 5;
  float bias[16];
#pragma unroll
  for (int j = 0; j < 16; j++) {
    const int ch = 16 * grp + j;
    bias[j] = (a.bias && ch < a.co_store) ? a.bias[ch] : 0.f;
  }
  int meta[PER];
  uint32_t qoff[PER];
#pragma unroll
  for (int q = 0; q < PER; q++) {
    meta[q] = halo_meta<CI, VS, SWZ>(threadIdx.x + q * NT);
    qoff[q] = a.qoff_ok ? halo_qoff<CI>(meta[q], a.D0, a.D1) : 0u;
  }
  for (int tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
    const TileXYZ t = tile_xyz(tile, a.nt0, a.nt1, a.nt2);
    uint4 pre[PER];
    fetch_halo<CI, WRAP, PER>(a, meta, qoff, t, pre);
    __syncthreads();  // the previous tile's reads of sh (and the weight copy) are done
#pragma unroll
    for (int q = 0; q < PER; q++)
      if (meta[q] >= 0) *reinterpret_cast<uint4 *>(sh + ((meta[q] >> 14) << 4)) = pre[q];
    __syncthreads();
    f32x16 acc[TY];
#pragma unroll
    for (int m = 0; m < TY; m++)
#pragma unroll
      for (int j = 0; j < 16; j++) acc[m][j] = 0.f;
#pragma unroll 1
    for (int tz = 0; tz < 3; tz++) {
#pragma unroll 1
      for (int tx = 0; tx < 3; tx++) {
        bf16x8 wa[3][KS];
#pragma unroll
        for (int ty = 0; ty < 3; ty++)
#pragma unroll
          for (int ks = 0; ks < KS; ks++)
            wa[ty][ks] = *reinterpret_cast<const bf16x8 *>(
                sw + (((9 * tz + 3 * ty + tx) * KS + ks) * 64 + lane) * 16);
        const int vrow = (wave + tz) * HY * HX + col + tx;
        const unsigned char *base = sh + vrow * VS + grp * 16;
#pragma unroll
        for (int hy = 0; hy < HY; hy++) {
#pragma unroll
          for (int ks = 0; ks < KS; ks++) {
            bf16x8 xb;
            if constexpr (SWZ) {
              const int vb = vrow + hy * HX;
              xb = *reinterpret_cast<const bf16x8 *>(sh + vb * VS + ((grp ^ ((vb >> 2) & 1)) << 4));
            } else {
              xb = *reinterpret_cast<const bf16x8 *>(base + hy * HX * VS + ks * 32);
            }
#pragma unroll
            for (int ty = 0; ty < 3; ty++) {
              const int my = hy - ty;
              if (my >= 0 && my < TY)
                acc[my] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wa[ty][ks], xb, acc[my], 0, 0, 0);
            }
          }
        }
      }
    }
    // epilogue: lane holds channels 16 grp .. 16 grp + 15 of voxel x = col
    const int oz = t.oz0 + wave, ox = t.ox0 + col;
#pragma unroll
    for (int my = 0; my < TY; my++) {
      const int oy = t.oy0 + my;
      if (oy >= a.E1 || oz >= a.E2 || ox >= a.E0) continue;
      const int64_t vox = (((int64_t)t.b * a.E2 + oz) * a.E1 + oy) * a.E0 + ox;
      float v[16];
#pragma unroll
      for (int j = 0; j < 16; j++) {
        v[j] = acc[my][j] + bias[j];
        if (a.relu) v[j] = fmaxf(v[j], 0.f);
      }
      if (VEC) {
        if (a.mask) {
          const uint4 *mp = reinterpret_cast<const uint4 *>(a.mask + vox * CO + 16 * grp);
          const uint4 m2[2] = {mp[0], mp[1]};
          const bf16 *mb = reinterpret_cast<const bf16 *>(m2);
#pragma unroll
          for (int j = 0; j < 16; j++)
            if (!((float)mb[j] > 0.f)) v[j] = 0.f;
        }
        bf16x8 o[2];
#pragma unroll
        for (int j = 0; j < 16; j++) o[j >> 3][j & 7] = (bf16)v[j];
        uint4 *yp = reinterpret_cast<uint4 *>(reinterpret_cast<bf16 *>(a.y) + vox * a.ystride + 16 * grp);
        yp[0] = *reinterpret_cast<const uint4 *>(&o[0]);
        yp[1] = *reinterpret_cast<const uint4 *>(&o[1]);
      } else {
#pragma unroll
        for (int j = 0; j < 16; j++) {
          const int ch = 16 * grp + j;
          if (ch >= a.co_store) continue;
          float w = v[j];
          if (a.mask && !((float)a.mask[vox * CO + ch] > 0.f)) w = 0.f;
          if (a.out_f32)
            reinterpret_cast<float *>(a.y)[vox * a.ystride + ch] = w;
          else
            reinterpret_cast<bf16 *>(a.y)[vox * a.ystride + ch] = (bf16)w;
        }
      }
    }
  }
}

// Narrow output (co <= 16, ci = 32): v_mfma_f32_16x16x32_bf16 computes 16
// output channels x 16 voxels with all 32 input channels in one instruction
// (lane l supplies A[row l%16][k 8(l/16)..+7] and B[k 8(l/16)..+7][col l%16];
// accumulator j of lane l is D[4(l/16) + j][l%16]), half the work of the
// 32-wide instruction for a layer with 3 real outputs.  The same transposed
// product, tiles, halo and row reuse as k_conv: the narrow packing is the A
// operand as it stands, and lane l ends with channels 4 (l/16) .. + 3 of
// voxel l%16 of each 16-voxel half of a row.  ADD: instead of storing the
// three outputs, add add_scale times each to the FP32 field add[c] at the
// output voxel (the closure's correction of the velocity components).
template <int WRAP, bool ADD>
__global__ __launch_bounds__(NT) void k_conv_n16(ConvArgs a) {
  constexpr int CI = 32;
  constexpr int VS = CI * 2 + 16;
  constexpr int NCHUNK = HX * HY * HZ * (CI / 8);
  constexpr int PER = (NCHUNK + NT - 1) / NT;
  __shared__ __align__(16) unsigned char sw[27 * 64 * 16];
  __shared__ __align__(16) unsigned char sh[HX * HY * HZ * VS];
  copy_weights<27 * 64, false>(sw, a.wp);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, grp = lane >> 4;
  float bias[4];
#pragma unroll
  for (int j = 0; j < 4; j++) {
    const int ch = 4 * grp + j;
    bias[j] = (a.bias && ch < a.co_store) ? a.bias[ch] : 0.f;
  }
  int meta[PER];
  uint32_t qoff[PER];
#pragma unroll
  for (int q = 0; q < PER; q++) {
    meta[q] = halo_meta<CI, VS>(threadIdx.x + q * NT);
    qoff[q] = a.qoff_ok ? halo_qoff<CI>(meta[q], a.D0, a.D1) : 0u;
  }
  for (int tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
    const TileXYZ t = tile_xyz(tile, a.nt0, a.nt1, a.nt2);
    uint4 pre[PER];
    fetch_halo<CI, WRAP, PER>(a, meta, qoff, t, pre);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; q++)
      if (meta[q] >= 0) *reinterpret_cast<uint4 *>(sh + ((meta[q] >> 14) << 4)) = pre[q];
    __syncthreads();
    f32x4 acc[TY][2];
#pragma unroll
    for (int m = 0; m < TY; m++)
#pragma unroll
      for (int h = 0; h < 2; h++)
#pragma unroll
        for (int j = 0; j < 4; j++) acc[m][h][j] = 0.f;
#pragma unroll 1
    for (int tz = 0; tz < 3; tz++) {
#pragma unroll 1
      for (int tx = 0; tx < 3; tx++) {
        bf16x8 wa[3];
#pragma unroll
        for (int ty = 0; ty < 3; ty++)
          wa[ty] = *reinterpret_cast<const bf16x8 *>(sw + ((9 * tz + 3 * ty + tx) * 64 + lane) * 16);
        const unsigned char *base = sh + ((wave + tz) * HY * HX + col + tx) * VS + grp * 16;
#pragma unroll
        for (int hy = 0; hy < HY; hy++) {
#pragma unroll
          for (int h = 0; h < 2; h++) {
            const bf16x8 xb = *reinterpret_cast<const bf16x8 *>(base + (hy * HX + 16 * h) * VS);
#pragma unroll
            for (int ty = 0; ty < 3; ty++) {
              const int my = hy - ty;
              if (my >= 0 && my < TY)
                acc[my][h] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[ty], xb, acc[my][h], 0, 0, 0);
            }
          }
        }
      }
    }
    const int oz = t.oz0 + wave;
    if (ADD) {
      // the lanes holding channels 0..2 (grp 0) add the outputs to the three
      // fields: every field value of the tile's rows is read before any is
      // written, so the reads are in flight together
      if (grp != 0) continue;
      float old[TY][2][3];
      int64_t at[TY][2];
#pragma unroll
      for (int my = 0; my < TY; my++)
#pragma unroll
        for (int h = 0; h < 2; h++) {
          const int oy = t.oy0 + my, ox = t.ox0 + 16 * h + col;
          const bool ok = oy < a.E1 && oz < a.E2 && ox < a.E0;
          at[my][h] = ok ? (((int64_t)t.b * a.E2 + oz) * a.E1 + oy) * a.E0 + ox : -1;
#pragma unroll
          for (int j = 0; j < 3; j++) old[my][h][j] = ok ? a.add[j][at[my][h]] : 0.f;
        }
#pragma unroll
      for (int my = 0; my < TY; my++)
#pragma unroll
        for (int h = 0; h < 2; h++) {
          if (at[my][h] < 0) continue;
#pragma unroll
          for (int j = 0; j < 3; j++) {
            float v = acc[my][h][j] + bias[j];
            if (a.relu) v = fmaxf(v, 0.f);
            a.add[j][at[my][h]] = __fmaf_rn(a.add_scale, v, old[my][h][j]);
          }
        }
      continue;
    }
#pragma unroll
    for (int my = 0; my < TY; my++) {
      const int oy = t.oy0 + my;
      if (oy >= a.E1 || oz >= a.E2) continue;
      const int64_t rowv = (((int64_t)t.b * a.E2 + oz) * a.E1 + oy) * a.E0;
#pragma unroll
      for (int h = 0; h < 2; h++) {
        const int ox = t.ox0 + 16 * h + col;
        if (ox >= a.E0) continue;
        const int64_t vox = rowv + ox;
#pragma unroll
        for (int j = 0; j < 4; j++) {
          const int ch = 4 * grp + j;
          if (ch >= a.co_store) continue;
          float v = acc[my][h][j] + bias[j];
          if (a.relu) v = fmaxf(v, 0.f);
          if (a.mask && !((float)a.mask[vox * CO + ch] > 0.f)) v = 0.f;
          if (a.out_f32)
            reinterpret_cast<float *>(a.y)[vox * a.ystride + ch] = v;
          else
            reinterpret_cast<bf16 *>(a.y)[vox * a.ystride + ch] = (bf16)v;
        }
      }
    }
  }
}

// ------------------------------------------------------ weight gradient --

struct WgradArgs {
  const bf16 *x;   // layer input [B][D..][CI]
  const bf16 *g;   // output gradient [B][E..][32]
  float *part;     // [gridDim][27*32*32 + 32]
  int B, D0, D1, D2, E0, E1, E2;
  int off, wrap;
  int nt0, nt1, nt2, ntiles;
};

// dW[t][ci][co] += sum over the tile's voxels p of x[p + t + off][ci] g[p][co]
// as [ci x 16 voxels] x [16 voxels x co] products; wave w owns the taps
// t = w, w + 4, ... (7 or 6 accumulators), wave 0 also sums g for the bias.
template <int CI>
__global__ __launch_bounds__(NT) void k_wgrad(WgradArgs a) {
  constexpr int VS = CI * 2 + 16;
  constexpr int GS = CO * 2 + 16;  // padded voxel stride of the gradient tile
  __shared__ __align__(16) unsigned char sh[HX * HY * HZ * VS];
  __shared__ __align__(16) unsigned char sg[TX * TY * TZ * GS];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row = lane & 31, grp = lane >> 5;
  f32x16 acc[7];
  for (int i = 0; i < 7; i++)
    for (int j = 0; j < 16; j++) acc[i][j] = 0.f;
  float bsum = 0.f;
  const int ntap = wave < 3 ? 7 : 6;
  for (int tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
    int r = tile;
    const int t0 = r % a.nt0;
    r /= a.nt0;
    const int t1 = r % a.nt1;
    r /= a.nt1;
    const int t2 = r % a.nt2;
    const int b = r / a.nt2;
    const int ox0 = t0 * TX, oy0 = t1 * TY, oz0 = t2 * TZ;
    __syncthreads();
    load_halo<CI, VS>(sh, a.x, b, ox0, oy0, oz0, a.D0, a.D1, a.D2, a.off, a.wrap);
    // gradient tile, zeros for voxels outside the output
    for (int c = threadIdx.x; c < TX * TY * TZ * 4; c += NT) {
      const int v = c >> 2, part = c & 3;
      const int vx = v % TX, vy = (v / TX) % TY, vz = v / (TX * TY);
      const int ox = ox0 + vx, oy = oy0 + vy, oz = oz0 + vz;
      uint4 val = make_uint4(0, 0, 0, 0);
      if (ox < a.E0 && oy < a.E1 && oz < a.E2) {
        const size_t vox = (((size_t)b * a.E2 + oz) * a.E1 + oy) * a.E0 + ox;
        val = *reinterpret_cast<const uint4 *>(a.g + vox * CO + part * 8);
      }
      *reinterpret_cast<uint4 *>(sg + v * GS + part * 16) = val;
    }
    __syncthreads();
#pragma unroll 1
    for (int s = 0; s < TX * TY * TZ / 16; s++) {
      // k-step s: 16 voxels of output row m = s / 2, x = (s % 2) 16 + 8 grp + e
      const int m = s >> 1, my = m % TY, mz = m / TY;
      const int xb = (s & 1) * 16 + 8 * grp;
      bf16x8 bg;
      const unsigned char *gp = sg + ((m * TX) + xb) * GS + row * 2;
#pragma unroll
      for (int e = 0; e < 8; e++) bg[e] = *reinterpret_cast<const bf16 *>(gp + e * GS);
      if (wave == 0)
#pragma unroll
        for (int e = 0; e < 8; e++) bsum += (float)bg[e];
#pragma unroll
      for (int i = 0; i < 7; i++) {
        if (i >= ntap) break;
        const int t = wave + 4 * i;
        const int tz = t / 9, ty = (t / 3) % 3, tx = t % 3;
        bf16x8 ax;
        if (row < CI) {
          const unsigned char *hp =
              sh + (((mz + tz) * HY + my + ty) * HX + xb + tx) * VS + row * 2;
#pragma unroll
          for (int e = 0; e < 8; e++) ax[e] = *reinterpret_cast<const bf16 *>(hp + e * VS);
        } else {
#pragma unroll
          for (int e = 0; e < 8; e++) ax[e] = (bf16)0.f;
        }
        acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ax, bg, acc[i], 0, 0, 0);
      }
    }
  }
  // partial sums of this workgroup: D[ci][co] of tap t
  float *out = a.part + (size_t)blockIdx.x * (27 * 32 * 32 + 32);
  for (int i = 0; i < ntap; i++) {
    const int t = wave + 4 * i;
#pragma unroll
    for (int j = 0; j < 16; j++) {
      const int ci = 8 * (j >> 2) + 4 * grp + (j & 3);
      out[(t * 32 + ci) * 32 + row] = acc[i][j];
    }
  }
  if (wave == 0) {
    bsum += __shfl_xor(bsum, 32);
    if (grp == 0) out[27 * 32 * 32 + row] = bsum;
  }
}

// dW[t][ci][co] (real sizes) = sum over workgroups of the partials; db too.
__global__ void k_wgrad_reduce(const float *part, int nblk, int ci, int co, float *dW,
                               float *db) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int nw = 27 * ci * co;
  if (i < nw) {
    const int c_o = i % co, c_i = (i / co) % ci, t = i / (co * ci);
    const size_t src = ((size_t)t * 32 + c_i) * 32 + c_o;
    float s = 0.f;
    for (int k = 0; k < nblk; k++) s += part[(size_t)k * (27 * 32 * 32 + 32) + src];
    dW[i] = s;
  } else if (i < nw + co) {
    const int c_o = i - nw;
    float s = 0.f;
    for (int k = 0; k < nblk; k++) s += part[(size_t)k * (27 * 32 * 32 + 32) + 27 * 32 * 32 + c_o];
    if (db) db[c_o] = s;
  }
}

// ------------------------------------------------------ small kernels --

// packed[t][ks][l][e] = W[t][ci = 16 ks + 8 (l/32) + e][co = l % 32] (0 outside);
// transposed: W'[t][c'][c''] = W[26 - t][c''][c'] with c' the input channel;
// narrow: packed[t][l][e] = W[t][ci = 8 (l/16) + e][co = l % 16].
__global__ void k_pack(const float *W, int ci, int co, int ci_pad, int transpose, bf16 *out) {
  const int KS = ci_pad / 16;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (transpose == IB_CONV_PACK_NARROW) {
    if (i >= 27 * 64 * 8) return;
    const int e = i & 7, l = (i >> 3) & 63, t = i >> 9;
    const int kin = 8 * (l >> 4) + e, kout = l & 15;
    out[i] = (bf16)((kin < ci && kout < co) ? W[((size_t)t * ci + kin) * co + kout] : 0.f);
    return;
  }
  if (i >= 27 * KS * 64 * 8) return;
  const int e = i & 7, l = (i >> 3) & 63, ks = (i >> 9) % KS, t = (i >> 9) / KS;
  const int kin = 16 * ks + 8 * (l >> 5) + e, kout = l & 31;
  float v = 0.f;
  if (!transpose) {
    if (kin < ci && kout < co) v = W[((size_t)t * ci + kin) * co + kout];
  } else {
    // adjoint: its input channel kin is the forward output channel, its output
    // channel kout the forward input channel
    if (kin < co && kout < ci) v = W[((size_t)(26 - t) * ci + kout) * co + kin];
  }
  out[i] = (bf16)v;
}

__global__ void k_mse(const float *pred, const float *target, int64_t nvox, int nch,
                      bf16 *grad, float *part) {
  __shared__ float red[256];
  const float sc = 2.f / (float)((double)nvox * nch);
  float s = 0.f;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nvox;
       v += (int64_t)gridDim.x * blockDim.x) {
    bf16x8 gv[4];
#pragma unroll
    for (int c = 0; c < 32; c++) {
      float g = 0.f;
      if (c < nch) {
        const float d = pred[v * nch + c] - target[v * nch + c];
        s += d * d;
        g = sc * d;
      }
      gv[c >> 3][c & 7] = (bf16)g;
    }
    for (int q = 0; q < 4; q++) reinterpret_cast<bf16x8 *>(grad + v * 32)[q] = gv[q];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_mse_finish(const float *part, int nblk, double denom, float *loss) {
  __shared__ float red[256];
  float s = 0.f;
  for (int i = threadIdx.x; i < nblk; i += blockDim.x) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = (float)(red[0] / denom);
}

__global__ void k_adam(float *th, const float *g, float *m, float *v, int64_t n, float lr,
                       float b1, float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

template <typename T>
__global__ void k_restrict(const T *f, int n0, int n1, int n2, int kind, T *c) {
  const int m0 = n0 / 2, m1 = n1 / 2, m2 = n2 / 2;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)m0 * m1 * m2) return;
  const int I = (int)(i % m0), J = (int)((i / m0) % m1), K = (int)(i / ((int64_t)m0 * m1));
  // spans along each axis: 2 fine indices, except 1 (index 2I) along a face's normal
  const int s0 = (kind == 0) ? 1 : 2, s1 = (kind == 1) ? 1 : 2, s2 = (kind == 2) ? 1 : 2;
  double acc = 0.0;
  for (int c = 0; c < s2; c++)
    for (int b = 0; b < s1; b++)
      for (int a = 0; a < s0; a++)
        acc += (double)f[((int64_t)(2 * K + c) * n1 + (2 * J + b)) * n0 + (2 * I + a)];
  c[i] = (T)(acc / (s0 * s1 * s2));
}

struct GatherArgs {
  const float *src[IB_GATHER_MAX_SOURCES];  // slots past nsrc repeat src[0]
  float scale[IB_GATHER_MAX_SOURCES];
  int chan[IB_GATHER_MAX_SOURCES];          // -1 past nsrc
  int n0, n1, n2;
  const int *origins;
  int B, d0, d1, d2, out_f32, out_ch;
  int slice_blocks;  // workgroups per brick slice (d0 d1 voxels)
  void *out;
};

// out[b][voxel][c] = sum over sources s with chan[s] = c of scale[s] src[s][g]
// at the periodic grid point g of the brick voxel (0 for channels no source
// names), the sources added in index order.  Workgroup w covers voxels of
// one brick slice (z, b) = w / slice_blocks, so only the in-slice position
// is divided per thread (32-bit); every source is loaded before any is used
// (a fixed number of loads, the spare slots reading source 0 again), so a
// thread's loads are in flight together.
__global__ void __launch_bounds__(256) k_gather(GatherArgs a) {
  const int slice = (int)blockIdx.x / a.slice_blocks;
  const int r = ((int)blockIdx.x - slice * a.slice_blocks) * 256 + (int)threadIdx.x;
  if (r >= a.d0 * a.d1) return;
  const int b = slice / a.d2, z = slice - b * a.d2;
  const int y = r / a.d0, x = r - y * a.d0;
  int gx = wrapi(a.origins[3 * b + 0], a.n0) + x;
  int gy = wrapi(a.origins[3 * b + 1], a.n1) + y;
  const int gz = wrapi(a.origins[3 * b + 2] + z, a.n2);
  if (gx >= a.n0) gx %= a.n0;
  if (gy >= a.n1) gy %= a.n1;
  const int64_t g = ((int64_t)gz * a.n1 + gy) * a.n0 + gx;
  float val[IB_GATHER_MAX_SOURCES];
#pragma unroll
  for (int s = 0; s < IB_GATHER_MAX_SOURCES; s++) val[s] = a.src[s][g];
  float v[16];
#pragma unroll
  for (int c = 0; c < 16; c++) v[c] = 0.f;
#pragma unroll
  for (int s = 0; s < IB_GATHER_MAX_SOURCES; s++) {
    const float t = val[s] * a.scale[s];
#pragma unroll
    for (int c = 0; c < 16; c++)
      if (c == a.chan[s]) v[c] += t;
  }
  const int64_t i = ((int64_t)slice * a.d1 + y) * a.d0 + x;
  if (a.out_f32) {
    float *o = reinterpret_cast<float *>(a.out) + i * a.out_ch;
#pragma unroll
    for (int c = 0; c < 16; c++)
      if (c < a.out_ch) o[c] = v[c];
  } else {
    bf16x8 w[2];
#pragma unroll
    for (int c = 0; c < 16; c++) w[c >> 3][c & 7] = (bf16)v[c];
    reinterpret_cast<bf16x8 *>(reinterpret_cast<bf16 *>(a.out) + i * 16)[0] = w[0];
    reinterpret_cast<bf16x8 *>(reinterpret_cast<bf16 *>(a.out) + i * 16)[1] = w[1];
  }
}

__global__ void k_apply(float *u0, float *u1, float *u2, int64_t nvox, const float *y, float s) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nvox) return;
  u0[i] = __fmaf_rn(s, y[3 * i + 0], u0[i]);
  u1[i] = __fmaf_rn(s, y[3 * i + 1], u1[i]);
  u2[i] = __fmaf_rn(s, y[3 * i + 2], u2[i]);
}

// ------------------------------------------------------------- host ----

using ibgm_err::fail;

#define HIP_CHECK_LAUNCH(what)                                                          \
  do {                                                                                  \
    hipError_t e_ = hipGetLastError();                                                  \
    if (e_ != hipSuccess) return fail(IB_E_DEVICE, "%s launch failed: %s", what,        \
                                      hipGetErrorString(e_));                           \
  } while (0)

ib_status mode_off(int32_t mode, int *off, int *wrap, int *grow) {
  switch (mode) {
    case IB_CONV_PERIODIC: *off = -1, *wrap = 1, *grow = 0; return IB_OK;
    case IB_CONV_VALID: *off = 0, *wrap = 0, *grow = -2; return IB_OK;
    case IB_CONV_FULL: *off = -2, *wrap = 0, *grow = 2; return IB_OK;
    default: return fail(IB_E_INVALID, "unknown convolution mode %d", mode);
  }
}

ib_status check_dims(const int32_t *d, int32_t batch, int grow, int64_t *nvox_in,
                     int64_t *nvox_out) {
  if (!d) return fail(IB_E_INVALID, "null dims");
  if (batch < 1) return fail(IB_E_INVALID, "batch < 1");
  int64_t vi = batch, vo = batch;
  for (int a = 0; a < 3; a++) {
    if (d[a] < 1 || d[a] > 4096) return fail(IB_E_INVALID, "dims[%d] = %d out of [1, 4096]", a, d[a]);
    if (d[a] + grow < 1) return fail(IB_E_INVALID, "dims[%d] = %d too small for a valid convolution", a, d[a]);
    vi *= d[a], vo *= d[a] + grow;
  }
  if (vi * 32 >= ((int64_t)1 << 40) || vo * 32 >= ((int64_t)1 << 40))
    return fail(IB_E_INVALID, "brick batch too large");
  *nvox_in = vi, *nvox_out = vo;
  return IB_OK;
}

ib_status launch_conv(const bf16 *x, int32_t batch, const int32_t *in_dims, int32_t ci_pad,
                      const void *packed, const float *bias, int32_t mode, int relu,
                      int out_f32, const bf16 *mask, void *y, int32_t co_store,
                      int32_t y_stride, hipStream_t st, bool narrow = false,
                      float *const *add = nullptr, float add_scale = 0.f) {
  int off, wrap, grow;
  ib_status s = mode_off(mode, &off, &wrap, &grow);
  if (s != IB_OK) return s;
  int64_t vi, vo;
  if ((s = check_dims(in_dims, batch, grow, &vi, &vo)) != IB_OK) return s;
  if (ci_pad != 16 && ci_pad != 32) return fail(IB_E_INVALID, "ci_pad must be 16 or 32");
  if (!x || !packed || !(y || add)) return fail(IB_E_INVALID, "null convolution buffer");
  if (co_store < 1 || co_store > CO || y_stride < co_store)
    return fail(IB_E_INVALID, "need 1 <= co_store <= 32 and y_stride >= co_store");
  if ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(packed)) & 15)
    return fail(IB_E_INVALID, "x and packed weights must be 16-byte aligned");
  ConvArgs a{};
  a.x = x, a.wp = reinterpret_cast<const bf16 *>(packed), a.bias = bias, a.mask = mask, a.y = y;
  a.B = batch, a.D0 = in_dims[0], a.D1 = in_dims[1], a.D2 = in_dims[2];
  a.E0 = a.D0 + grow, a.E1 = a.D1 + grow, a.E2 = a.D2 + grow;
  a.off = off, a.wrap = wrap, a.relu = relu, a.out_f32 = out_f32;
  a.co_store = co_store, a.ystride = y_stride;
  if (add) {
    for (int c = 0; c < 3; c++) a.add[c] = add[c];
    a.add_scale = add_scale;
  }
  a.nt0 = (a.E0 + TX - 1) / TX, a.nt1 = (a.E1 + TY - 1) / TY, a.nt2 = (a.E2 + TZ - 1) / TZ;
  const int64_t nt = (int64_t)a.nt0 * a.nt1 * a.nt2 * batch;
  if (nt >= INT32_MAX) return fail(IB_E_INVALID, "too many tiles");
  a.ntiles = (int)nt;
  a.qoff_ok = (int64_t)HZ * a.D1 * a.D0 * (ci_pad * 2) < ((int64_t)1 << 31);
  // two resident workgroups per CU for the 16-channel kernel (its LDS fits twice)
  const int64_t wg = (!narrow && ci_pad == 16) ? 2 * WG_CONV : WG_CONV;
  const int grid = (int)(nt < wg ? nt : wg);
  if (wrap && (a.D0 < HX || a.D1 < HY || a.D2 < HZ)) a.wrap = 2;
  // 16-byte output stores: 32 BF16 channels per voxel at a stride that keeps
  // every voxel's record 16-byte aligned (and the mask, when given)
  const bool vec = !narrow && !out_f32 && co_store == CO && y_stride % 8 == 0 &&
                   !(reinterpret_cast<uintptr_t>(y) & 15) &&
                   !(reinterpret_cast<uintptr_t>(mask) & 15);
  auto go = [&](auto wrap_tag) {
    constexpr int W = decltype(wrap_tag)::value;
    if (add) k_conv_n16<W, true><<<grid, NT, 0, st>>>(a);
    else if (narrow) k_conv_n16<W, false><<<grid, NT, 0, st>>>(a);
    else if (ci_pad == 16) {
      if (vec) k_conv<16, W, true><<<grid, NT, 0, st>>>(a);
      else k_conv<16, W, false><<<grid, NT, 0, st>>>(a);
    } else {
      if (vec) k_conv<32, W, true><<<grid, NT, 0, st>>>(a);
      else k_conv<32, W, false><<<grid, NT, 0, st>>>(a);
    }
  };
  if (a.wrap == 1) go(std::integral_constant<int, 1>{});
  else if (a.wrap == 2) go(std::integral_constant<int, 2>{});
  else go(std::integral_constant<int, 0>{});
  HIP_CHECK_LAUNCH("conv3d");
  return IB_OK;
}

}  // namespace

extern "C" ib_status ib_conv3d_pack(const float *W, int32_t ci, int32_t co, int32_t ci_pad,
                                    int32_t transpose, void *packed, void *hip_stream) {
  if (!W || !packed) return fail(IB_E_INVALID, "null weights");
  if (ci_pad != 16 && ci_pad != 32) return fail(IB_E_INVALID, "ci_pad must be 16 or 32");
  if (ci < 1 || co < 1 || co > 32 || ci > 32)
    return fail(IB_E_INVALID, "channels out of range (ci %d, co %d)", ci, co);
  if (transpose < 0 || transpose > IB_CONV_PACK_NARROW) return fail(IB_E_INVALID, "unknown packing %d", transpose);
  if (transpose != 1 && ci > ci_pad) return fail(IB_E_INVALID, "ci > ci_pad");
  if (transpose && ci_pad != 32) return fail(IB_E_INVALID, "the adjoint and narrow packings need ci_pad 32");
  if (transpose == IB_CONV_PACK_NARROW && co > 16) return fail(IB_E_INVALID, "the narrow packing needs co <= 16");
  const int n = transpose == IB_CONV_PACK_NARROW ? 27 * 64 * 8 : 27 * (ci_pad / 16) * 64 * 8;
  k_pack<<<(n + 255) / 256, 256, 0, (hipStream_t)hip_stream>>>(W, ci, co, ci_pad, transpose,
                                                                reinterpret_cast<bf16 *>(packed));
  HIP_CHECK_LAUNCH("pack");
  return IB_OK;
}

extern "C" ib_status ib_conv3d_fwd(const uint16_t *x, int32_t batch, const int32_t in_dims[3],
                                   int32_t ci_pad, const void *packed, const float *bias,
                                   int32_t mode, int32_t flags, void *y, int32_t co_store,
                                   int32_t y_stride, void *hip_stream) {
  if (flags & ~(IB_CONV_RELU | IB_CONV_OUT_F32 | IB_CONV_NARROW))
    return fail(IB_E_INVALID, "unknown flags");
  if ((flags & IB_CONV_NARROW) && (ci_pad != 32 || co_store > 16))
    return fail(IB_E_INVALID, "IB_CONV_NARROW needs ci_pad 32 and co_store <= 16");
  return launch_conv(reinterpret_cast<const bf16 *>(x), batch, in_dims, ci_pad, packed, bias,
                     mode, (flags & IB_CONV_RELU) != 0, (flags & IB_CONV_OUT_F32) != 0, nullptr,
                     y, co_store, y_stride, (hipStream_t)hip_stream,
                     (flags & IB_CONV_NARROW) != 0);
}

extern "C" ib_status ib_conv3d_bwd_data(const uint16_t *gy, int32_t batch,
                                        const int32_t out_dims[3], const void *packed,
                                        int32_t mode, const uint16_t *act_below, uint16_t *gx,
                                        void *hip_stream) {
  int32_t amode;
  if (mode == IB_CONV_PERIODIC) amode = IB_CONV_PERIODIC;
  else if (mode == IB_CONV_VALID) amode = IB_CONV_FULL;
  else return fail(IB_E_INVALID, "bwd_data: the layer must have run PERIODIC or VALID");
  return launch_conv(reinterpret_cast<const bf16 *>(gy), batch, out_dims, 32, packed, nullptr,
                     amode, 0, 0, reinterpret_cast<const bf16 *>(act_below), gx, 32, 32,
                     (hipStream_t)hip_stream);
}

extern "C" ib_status ib_conv3d_bwd_weight(const uint16_t *x, const uint16_t *gy, int32_t batch,
                                          const int32_t in_dims[3], int32_t ci_pad,
                                          int32_t mode, int32_t ci, int32_t co, float *dW,
                                          float *db, void *workspace, void *hip_stream) {
  int off, wrap, grow;
  ib_status s = mode_off(mode, &off, &wrap, &grow);
  if (s != IB_OK) return s;
  if (mode == IB_CONV_FULL) return fail(IB_E_INVALID, "bwd_weight: FULL layers are not built");
  int64_t vi, vo;
  if ((s = check_dims(in_dims, batch, grow, &vi, &vo)) != IB_OK) return s;
  if (ci_pad != 16 && ci_pad != 32) return fail(IB_E_INVALID, "ci_pad must be 16 or 32");
  if (ci < 1 || ci > ci_pad || co < 1 || co > 32) return fail(IB_E_INVALID, "channels out of range");
  if (!x || !gy || !dW || !workspace) return fail(IB_E_INVALID, "null buffer");
  if ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(gy) |
       reinterpret_cast<uintptr_t>(workspace)) & 15)
    return fail(IB_E_INVALID, "x, gy and workspace must be 16-byte aligned");
  hipStream_t st = (hipStream_t)hip_stream;
  WgradArgs a{};
  a.x = reinterpret_cast<const bf16 *>(x), a.g = reinterpret_cast<const bf16 *>(gy);
  a.part = reinterpret_cast<float *>(workspace);
  a.B = batch, a.D0 = in_dims[0], a.D1 = in_dims[1], a.D2 = in_dims[2];
  a.E0 = a.D0 + grow, a.E1 = a.D1 + grow, a.E2 = a.D2 + grow;
  a.off = off, a.wrap = wrap;
  a.nt0 = (a.E0 + TX - 1) / TX, a.nt1 = (a.E1 + TY - 1) / TY, a.nt2 = (a.E2 + TZ - 1) / TZ;
  const int64_t nt = (int64_t)a.nt0 * a.nt1 * a.nt2 * batch;
  if (nt >= INT32_MAX) return fail(IB_E_INVALID, "too many tiles");
  a.ntiles = (int)nt;
  const int grid = (int)(nt < IB_CONV_WGRAD_BLOCKS ? nt : IB_CONV_WGRAD_BLOCKS);
  if (ci_pad == 16) k_wgrad<16><<<grid, NT, 0, st>>>(a);
  else k_wgrad<32><<<grid, NT, 0, st>>>(a);
  HIP_CHECK_LAUNCH("wgrad");
  const int nout = 27 * ci * co + co;
  k_wgrad_reduce<<<(nout + 255) / 256, 256, 0, st>>>(a.part, grid, ci, co, dW, db);
  HIP_CHECK_LAUNCH("wgrad reduce");
  return IB_OK;
}

extern "C" ib_status ib_mse_grad(const float *pred, const float *target, int64_t n_vox,
                                 int32_t nch, float *loss, uint16_t *grad, void *workspace,
                                 void *hip_stream) {
  if (!pred || !target || !loss || !grad || !workspace) return fail(IB_E_INVALID, "null buffer");
  if (n_vox < 1 || nch < 1 || nch > 32) return fail(IB_E_INVALID, "bad n_vox / nch");
  if (reinterpret_cast<uintptr_t>(grad) & 15) return fail(IB_E_INVALID, "grad must be 16-byte aligned");
  hipStream_t st = (hipStream_t)hip_stream;
  const int64_t want = (n_vox + 255) / 256;
  const int nblk = (int)(want < 1024 ? want : 1024);
  float *part = reinterpret_cast<float *>(workspace);
  k_mse<<<nblk, 256, 0, st>>>(pred, target, n_vox, nch, reinterpret_cast<bf16 *>(grad), part);
  HIP_CHECK_LAUNCH("mse");
  k_mse_finish<<<1, 256, 0, st>>>(part, nblk, (double)n_vox * nch, loss);
  HIP_CHECK_LAUNCH("mse finish");
  return IB_OK;
}

extern "C" ib_status ib_adam_step(float *theta, const float *g, float *m, float *v, int64_t n,
                                  float lr, float beta1, float beta2, float eps, int32_t t,
                                  void *hip_stream) {
  if (!theta || !g || !m || !v) return fail(IB_E_INVALID, "null buffer");
  if (n < 1 || t < 1) return fail(IB_E_INVALID, "need n >= 1 and t >= 1");
  if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps > 0.f && lr >= 0.f))
    return fail(IB_E_INVALID, "bad Adam hyper-parameters");
  const float c1 = 1.f - (float)std::pow((double)beta1, (double)t);
  const float c2 = 1.f - (float)std::pow((double)beta2, (double)t);
  k_adam<<<(unsigned)((n + 255) / 256), 256, 0, (hipStream_t)hip_stream>>>(theta, g, m, v, n, lr,
                                                                           beta1, beta2, eps, c1, c2);
  HIP_CHECK_LAUNCH("adam");
  return IB_OK;
}

extern "C" ib_status ib_restrict(const void *fine, int32_t dtype, const int32_t nf[3],
                                 int32_t kind, void *coarse, void *hip_stream) {
  if (!fine || !coarse || !nf) return fail(IB_E_INVALID, "null buffer");
  if (kind < 0 || kind > 3) return fail(IB_E_INVALID, "kind must be 0..3");
  for (int a = 0; a < 3; a++)
    if (nf[a] < 2 || nf[a] % 2 || nf[a] > 4096) return fail(IB_E_INVALID, "nf[%d] must be even in [2, 4096]", a);
  const int64_t nc = (int64_t)(nf[0] / 2) * (nf[1] / 2) * (nf[2] / 2);
  hipStream_t st = (hipStream_t)hip_stream;
  const unsigned g = (unsigned)((nc + 255) / 256);
  if (dtype == IB_F64)
    k_restrict<double><<<g, 256, 0, st>>>((const double *)fine, nf[0], nf[1], nf[2], kind, (double *)coarse);
  else if (dtype == IB_F32)
    k_restrict<float><<<g, 256, 0, st>>>((const float *)fine, nf[0], nf[1], nf[2], kind, (float *)coarse);
  else
    return fail(IB_E_INVALID, "unknown dtype %d", dtype);
  HIP_CHECK_LAUNCH("restrict");
  return IB_OK;
}

extern "C" ib_status ib_closure_gather(const float *const *src, const float *scales,
                                       const int32_t *chan, int32_t nsrc, const int32_t n[3],
                                       const int32_t *origins, int32_t batch,
                                       const int32_t dims[3], int32_t out_f32, int32_t out_ch,
                                       void *out, void *hip_stream) {
  if (!src || !scales || !chan || !n || !origins || !dims || !out)
    return fail(IB_E_INVALID, "null argument");
  if (nsrc < 1 || nsrc > IB_GATHER_MAX_SOURCES)
    return fail(IB_E_INVALID, "nsrc must be 1..%d", IB_GATHER_MAX_SOURCES);
  if (batch < 1) return fail(IB_E_INVALID, "batch < 1");
  if (out_f32 ? (out_ch < 1 || out_ch > 16) : out_ch != 16)
    return fail(IB_E_INVALID, "out_ch must be 16 (BF16) or 1..16 (FP32)");
  GatherArgs a{};
  for (int s = 0; s < nsrc; s++) {
    if (!src[s]) return fail(IB_E_INVALID, "null source %d", s);
    if (chan[s] < 0 || chan[s] >= out_ch) return fail(IB_E_INVALID, "chan[%d] out of range", s);
    a.src[s] = src[s], a.scale[s] = scales[s], a.chan[s] = chan[s];
  }
  for (int s = nsrc; s < IB_GATHER_MAX_SOURCES; s++) a.src[s] = src[0], a.scale[s] = 0.f, a.chan[s] = -1;
  for (int i = 0; i < 3; i++)
    if (n[i] < 1 || dims[i] < 1 || n[i] > 4096 || dims[i] > 4096) return fail(IB_E_INVALID, "bad n / dims");
  if (!out_f32 && (reinterpret_cast<uintptr_t>(out) & 15)) return fail(IB_E_INVALID, "out must be 16-byte aligned");
  a.n0 = n[0], a.n1 = n[1], a.n2 = n[2], a.origins = origins;
  a.B = batch, a.d0 = dims[0], a.d1 = dims[1], a.d2 = dims[2], a.out_f32 = out_f32 ? 1 : 0;
  a.out_ch = out_ch, a.out = out;
  a.slice_blocks = (dims[0] * dims[1] + 255) / 256;
  const int64_t blocks = (int64_t)a.slice_blocks * dims[2] * batch;
  if (blocks > INT32_MAX) return fail(IB_E_INVALID, "gather batch too large");
  k_gather<<<(unsigned)blocks, 256, 0, (hipStream_t)hip_stream>>>(a);
  HIP_CHECK_LAUNCH("gather");
  return IB_OK;
}

extern "C" ib_status ib_closure_apply(float *const u[3], const int32_t n[3], const float *y,
                                      float scale, void *hip_stream) {
  if (!u || !n || !y || !u[0] || !u[1] || !u[2]) return fail(IB_E_INVALID, "null argument");
  for (int i = 0; i < 3; i++)
    if (n[i] < 1 || n[i] > 4096) return fail(IB_E_INVALID, "bad n");
  const int64_t nv = (int64_t)n[0] * n[1] * n[2];
  k_apply<<<(unsigned)((nv + 255) / 256), 256, 0, (hipStream_t)hip_stream>>>(u[0], u[1], u[2], nv, y, scale);
  HIP_CHECK_LAUNCH("apply");
  return IB_OK;
}

extern "C" ib_status ib_closure_conv_apply(const uint16_t *x, const int32_t n[3],
                                           const void *packed, const float *bias, float scale,
                                           float *const u[3], void *hip_stream) {
  if (!u || !u[0] || !u[1] || !u[2]) return fail(IB_E_INVALID, "null velocity component");
  if (u[0] == u[1] || u[0] == u[2] || u[1] == u[2])
    return fail(IB_E_INVALID, "the three velocity components must be distinct arrays");
  if (!std::isfinite(scale)) return fail(IB_E_INVALID, "scale is not finite");
  return launch_conv(reinterpret_cast<const bf16 *>(x), 1, n, 32, packed, bias,
                     IB_CONV_PERIODIC, 0, 1, nullptr, nullptr, 3, 3, (hipStream_t)hip_stream,
                     true, u, scale);
}
