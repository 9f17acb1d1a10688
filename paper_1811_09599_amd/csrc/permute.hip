// Binary index permutations of complex64 tensors (plain, and into the split layouts).
#include "kernel_util.h"

namespace qflex {
namespace dev {

// =============================================================================================
// Binary index permutation (paper, Methods B.2: reordering so that contracted indexes are
// contiguous for the matrix product).  GPU form: each workgroup moves one tile of 2^tile_bits
// elements through LDS.  The tile holds the lowest input bits (so every read is a run of
// consecutive addresses) and the lowest output bits (so every write is too); the remaining
// bits enumerate tiles.  A permutation that keeps the low bits in place degenerates into a
// block copy.
// =============================================================================================
PermTile make_perm_tile(int nbits, const int* perm) {
  if (nbits > kPermMaxBits) throw std::runtime_error("permute: too many index bits");
  PermTile t{};
  t.nbits = nbits;
  int inv[kPermMaxBits];
  for (int j = 0; j < nbits; ++j) inv[perm[j]] = j;
  const int T = std::min(nbits, kPermMaxTile);
  bool in_tile[kPermMaxBits] = {false};
  int size = 0;
  for (int p = 0; p < std::min(nbits, 5); ++p) in_tile[p] = true, ++size;
  for (int j = 0; j < nbits && size < T; ++j)
    if (!in_tile[perm[j]]) in_tile[perm[j]] = true, ++size;
  for (int p = 0; p < nbits && size < T; ++p)
    if (!in_tile[p]) in_tile[p] = true, ++size;
  t.tile_bits = size;
  int ti = 0;
  int read_index_of[kPermMaxBits];
  for (int p = 0; p < nbits; ++p)
    if (in_tile[p]) read_index_of[p] = ti, t.tile_in[ti++] = (int8_t)p;
  // write order: tile bits by output position
  int to = 0;
  for (int j = 0; j < nbits; ++j)
    if (in_tile[perm[j]]) {
      t.tile_out[to] = (int8_t)j;
      t.j2i[to] = (int8_t)read_index_of[perm[j]];
      ++to;
    }
  int r = 0;
  for (int p = 0; p < nbits; ++p)
    if (!in_tile[p]) {
      t.rest_in[r] = (int8_t)p;
      t.rest_out[r] = (int8_t)inv[p];
      ++r;
    }
  t.nrest = r;
  return t;
}


__global__ void __launch_bounds__(256) permute_kernel(const float2* __restrict__ in,
                                                      float2* __restrict__ out,
                                                      const PermTile t) {
  __shared__ float2 tile[(1 << kPermMaxTile) + (1 << kPermMaxTile) / 32];
  const int64_t batch_stride = int64_t(1) << t.nbits;
  in += (int64_t)blockIdx.y * batch_stride;
  out += (int64_t)blockIdx.y * batch_stride;
  const int64_t T = blockIdx.x;
  const int64_t in_base = rest_offset(T, t.rest_in, t.nrest);
  const int64_t out_base = rest_offset(T, t.rest_out, t.nrest);
  const int tb = t.tile_bits;
  const int tsize = 1 << tb;
  const int tid = threadIdx.x;
  const int nk = tsize > 256 ? tsize >> 8 : 1;
  if (tid < tsize) {
    const int64_t in_lo = in_base + deposit<0, 8>(tid, t.tile_in, tb);
    for (int k = 0; k < nk; ++k)
      tile[lds_pad(tid + (k << 8))] = in[in_lo + deposit<8, kPermMaxTile>(k, t.tile_in, tb)];
  }
  __syncthreads();
  if (tid < tsize) {
    const int i_lo = deposit_i<0, 8>(tid, t.j2i, tb);
    const int64_t out_lo = out_base + deposit<0, 8>(tid, t.tile_out, tb);
    for (int k = 0; k < nk; ++k) {
      const int i = i_lo | deposit_i<8, kPermMaxTile>(k, t.j2i, tb);
      out[out_lo + deposit<8, kPermMaxTile>(k, t.tile_out, tb)] = tile[lds_pad(i)];
    }
  }
}

void permute(const float2* in, float2* out, int64_t batch, const PermTile& t, hipStream_t s) {
  const int64_t tiles = int64_t(1) << t.nrest;
  if (batch < 1 || batch > 65535) throw std::runtime_error("permute: bad batch");
  hipLaunchKernelGGL(permute_kernel, dim3((unsigned)tiles, (unsigned)batch), dim3(256), 0, s, in,
                     out, t);
  check_launch("permute");
}

// =============================================================================================
// Split layouts of the 16-bit products (see kernels.h for the layout and the two formats).
// =============================================================================================
// One thread per group of 4 consecutive k of a row: the tile's write order starts with the
// lowest output bits, so a group is 4 consecutive write indices and is stored as two 16-byte
// vectors.  For fp16, every value is first multiplied by the operand's power-of-two scale,
// derived from the largest magnitude that absmax() recorded in *amax.
template <bool F16>
__global__ void __launch_bounds__(256) split_permute_kernel(const float2* __restrict__ in,
                                                            uint16_t* __restrict__ out,
                                                            const PermTile t,
                                                            const uint64_t* __restrict__ amax) {
  __shared__ float2 tile[(1 << kPermMaxTile) + (1 << kPermMaxTile) / 32];
  const int64_t n_el = int64_t(1) << t.nbits;
  in += (int64_t)blockIdx.y * n_el;
  out += (int64_t)blockIdx.y * n_el * 4;
  const int64_t T = blockIdx.x;
  const int64_t in_base = rest_offset(T, t.rest_in, t.nrest);
  const int64_t out_base = rest_offset(T, t.rest_out, t.nrest);
  const int tb = t.tile_bits;
  const int tsize = 1 << tb;
  const int tid = threadIdx.x;
  const int nk = tsize > 256 ? tsize >> 8 : 1;
  if (tid < tsize) {
    const int64_t in_lo = in_base + deposit<0, 8>(tid, t.tile_in, tb);
    for (int k = 0; k < nk; ++k)
      tile[lds_pad(tid + (k << 8))] = in[in_lo + deposit<8, kPermMaxTile>(k, t.tile_in, tb)];
  }
  float scale = 1.f;
  if constexpr (F16) scale = fp16_scale(*amax);
  __syncthreads();
  // group q holds write indices 4q..4q+3 (write bits 0 and 1 are the two lowest k bits);
  // a tile of up to 1024 elements has at most 256 groups
  const int ngroups = tsize >> 2;
  if (tid < ngroups) {
    const int q = tid;
    // write index bits 2.. come from q
    int ig = 0;
    int64_t e0 = out_base;
#pragma unroll
    for (int b = 2; b < kPermMaxTile; ++b)
      if (b < tb) {
        const int bit = (q >> (b - 2)) & 1;
        ig |= bit << t.j2i[b];
        e0 |= (int64_t)bit << t.tile_out[b];
      }
    float re[4], im[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = ig | ((u & 1) << t.j2i[0]) | (((u >> 1) & 1) << t.j2i[1]);
      const float2 v = tile[lds_pad(i)];
      re[u] = v.x * scale;
      im[u] = v.y * scale;
    }
    uint4 v0, v1;  // [rh, ih] and [rl, il] of the 4 k
    split16x2<F16>(re[0], re[1], v0.x, v1.x);
    split16x2<F16>(re[2], re[3], v0.y, v1.y);
    split16x2<F16>(im[0], im[1], v0.z, v1.z);
    split16x2<F16>(im[2], im[3], v0.w, v1.w);
    uint4* o = reinterpret_cast<uint4*>(out + 4 * e0);  // e0 is a multiple of 4
    o[0] = v0;
    o[1] = v1;
  }
}

void split_permute(const float2* in, uint16_t* out, int64_t batch, const PermTile& t, int kbits,
                   const uint64_t* amax, hipStream_t s) {
  if (batch < 1 || batch > 65535) throw std::runtime_error("split_permute: bad batch");
  // a thread's 4 consecutive write indices must be the 4 lowest k of one row
  if (kbits < 2 || t.tile_bits < 2 || t.tile_out[0] != 0 || t.tile_out[1] != 1)
    throw std::runtime_error("split_permute: K must be >= 4 and the tile must hold the 2 lowest bits");
  const int64_t tiles = int64_t(1) << t.nrest;
  if (amax)
    hipLaunchKernelGGL(split_permute_kernel<true>, dim3((unsigned)tiles, (unsigned)batch),
                       dim3(256), 0, s, in, out, t, amax);
  else
    hipLaunchKernelGGL(split_permute_kernel<false>, dim3((unsigned)tiles, (unsigned)batch),
                       dim3(256), 0, s, in, out, t, amax);
  check_launch("split_permute");
}

// Largest magnitude of the real and imaginary parts of n complex values, recorded as
// (tag << 32 | float bits) by a 64-bit atomic maximum: non-negative floats order like their
// bit patterns, and a larger tag replaces whatever an earlier call left in the slot.
__global__ void __launch_bounds__(256) absmax_kernel(const float4* __restrict__ in, int64_t n4,
                                                     const float2* __restrict__ tail,
                                                     uint64_t* __restrict__ slot, uint64_t tag) {
  float m = 0.f;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  // four independent loads in flight per thread
  for (; i + 3 * stride < n4; i += 4 * stride) {
    f32x4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = *reinterpret_cast<const f32x4*>(in + i + u * stride);
#pragma unroll
    for (int u = 0; u < 4; ++u)
      m = fmaxf(m, fmaxf(fmaxf(fabsf(v[u].x), fabsf(v[u].y)), fmaxf(fabsf(v[u].z), fabsf(v[u].w))));
  }
  for (; i < n4; i += stride) {
    const f32x4 v = *reinterpret_cast<const f32x4*>(in + i);
    m = fmaxf(m, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
  }
  if (tail && blockIdx.x == 0 && threadIdx.x == 0) m = fmaxf(m, fmaxf(fabsf(tail->x), fabsf(tail->y)));
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0)
    atomicMax(reinterpret_cast<unsigned long long*>(slot),
              (unsigned long long)(tag | __float_as_uint(m)));
}

void absmax(const float2* in, int64_t n, uint64_t* slot, uint32_t tag, hipStream_t s) {
  if (n < 1) throw std::runtime_error("absmax: empty input");
  if (tag == 0) throw std::runtime_error("absmax: tag must be non-zero");
  if (reinterpret_cast<uintptr_t>(in) % 16) throw std::runtime_error("absmax: misaligned input");
  const int64_t n4 = n / 2;
  const float2* tail = (n & 1) ? in + (n - 1) : nullptr;
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((n4 + 1023) / 1024, 4096));
  hipLaunchKernelGGL(absmax_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                     reinterpret_cast<const float4*>(in), n4, tail, slot,
                     (uint64_t)tag << 32);
  check_launch("absmax");
}

struct PermBits {
  int8_t p[kPermMaxBits];
};

__global__ void scatter_add_perm_kernel(const float2* __restrict__ in, int nbits, PermBits pb,
                                        double2* __restrict__ out, const int64_t* __restrict__ off,
                                        int64_t add) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = int64_t(1) << nbits;
  if (e >= n) return;
  const int b = blockIdx.y;
  int64_t o = 0;
  for (int j = 0; j < nbits; ++j) o |= ((e >> pb.p[j]) & 1) << j;
  const float2 v = in[(int64_t)b * n + e];
  double2* dst = out + add + (off ? off[b] : 0) + o;
  atomicAdd(&dst->x, (double)v.x);
  atomicAdd(&dst->y, (double)v.y);
}

void scatter_add_perm(const float2* in, int nbits, const int8_t* perm, int batch, double2* out,
                      const int64_t* off, int64_t add, hipStream_t s) {
  if (nbits > kPermMaxBits) throw std::runtime_error("scatter_add_perm: too many bits");
  PermBits pb{};
  for (int j = 0; j < nbits; ++j) pb.p[j] = perm[j];
  const int64_t n = int64_t(1) << nbits;
  hipLaunchKernelGGL(scatter_add_perm_kernel, dim3((unsigned)((n + 255) / 256), (unsigned)batch),
                     dim3(256), 0, s, in, nbits, pb, out, off, add);
  check_launch("scatter_add_perm");
}
}  // namespace dev
}  // namespace qflex
