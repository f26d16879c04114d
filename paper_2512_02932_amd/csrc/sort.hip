// Integer stages of the tile pipeline, gfx950: exclusive scan, gather,
// duplicate, stable LSD radix sort of (u32 key, u32 value) pairs, tile-range
// identification and fills.
//
// The (tile, depth) order of the pairs is reached in two sorts.  The V*N
// splat instances are sorted by their 32-bit depth key first (values are
// instance ids, so equal depths keep index order); the pairs are then
// duplicated in that order and stably sorted by tile id alone.  The result
// equals one stable sort of the 64-bit keys (tile << 32 | depth) of pairs
// duplicated in index order, with far fewer bits sorted per pair.
//
// The radix sort uses 8-bit digits.  A pass is three launches over
// fixed-size chunks of 4096 pairs:
//   * a per-chunk digit histogram (LDS atomics);
//   * an exclusive scan of the histogram table in digit-major order;
//   * a stable scatter.
// Within a chunk, elements are ranked in input order 256 at a time.  Each
// wave64 matches equal digits with 8 ballots, the four waves are combined in
// LDS, and a running per-digit base carries the count across rounds.
// Stability across chunks follows from the digit-major scan.

#include "hgs_internal.h"

namespace hgs {

namespace {

constexpr int kScanItems = 16;                       // elements per thread
constexpr int kScanChunk = kBlock * kScanItems;      // 4096 per block
constexpr int64_t kFlatChunks = 2048;  // up to 8M elements: two launches per scan

// Element count of a launch: the host capacity n, or min(n, *n_dev) when the
// count lives on the device (graph-captured launches never read it back).
__device__ __forceinline__ int64_t eff_n(int64_t n, const uint64_t *n_dev) {
  if (!n_dev) return n;
  const uint64_t d = *n_dev;
  return d < (uint64_t)n ? (int64_t)d : n;
}

// ----- block-wide exclusive scan of one value per thread (256 threads) -----
template <typename T>
__device__ inline T block_exclusive_scan(T v, T *lds, T &total) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  // inclusive scan within the wave
  T x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    T y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) lds[w] = x;
  __syncthreads();
  T off = 0;
  T tot = 0;
#pragma unroll
  for (int k = 0; k < kBlock / 64; ++k) {
    const T t = lds[k];
    if (k < w) off += t;
    tot += t;
  }
  __syncthreads();
  total = tot;
  return off + x - v;
}

// Level 0: per-chunk sums (u64) of u32 input.
__global__ void __launch_bounds__(256) scan_reduce_u32(const uint32_t *__restrict__ in, int64_t n,
                                                       const uint64_t *__restrict__ n_dev,
                                                       uint64_t *__restrict__ sums) {
  __shared__ uint64_t lds[4];
  n = eff_n(n, n_dev);
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  uint64_t acc = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + (int64_t)k * kBlock + threadIdx.x;
    if (i < n) acc += in[i];
  }
  uint64_t tot;
  block_exclusive_scan<uint64_t>(acc, lds, tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(256) scan_reduce_u64(const uint64_t *__restrict__ in, int64_t n,
                                                       uint64_t *__restrict__ sums) {
  __shared__ uint64_t lds[4];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  uint64_t acc = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + (int64_t)k * kBlock + threadIdx.x;
    if (i < n) acc += in[i];
  }
  uint64_t tot;
  block_exclusive_scan<uint64_t>(acc, lds, tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// Exclusive scan of one chunk in place given the chunk's offset.  Each
// thread owns kScanItems consecutive elements.
template <typename TI, typename TO>
__device__ inline void scan_chunk(const TI *in, TO *out, int64_t n, uint64_t offset,
                                  uint64_t *lds) {
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
  uint64_t vals[kScanItems];
  uint64_t acc = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + k;
    vals[k] = i < n ? (uint64_t)in[i] : 0;
    acc += vals[k];
  }
  uint64_t tot;
  uint64_t run = block_exclusive_scan<uint64_t>(acc, lds, tot) + offset;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + k;
    if (i < n) out[i] = (TO)run;
    run += vals[k];
  }
}

__global__ void __launch_bounds__(256) scan_down_u32(const uint32_t *__restrict__ in,
                                                     uint32_t *__restrict__ out, int64_t n,
                                                     const uint64_t *__restrict__ n_dev,
                                                     const uint64_t *__restrict__ offs) {
  __shared__ uint64_t lds[4];
  n = eff_n(n, n_dev);
  if ((int64_t)blockIdx.x * kScanChunk >= n) return;
  scan_chunk<uint32_t, uint32_t>(in, out, n, offs ? offs[blockIdx.x] : 0, lds);
}

__global__ void __launch_bounds__(256) scan_down_u64(const uint64_t *__restrict__ in,
                                                     uint64_t *__restrict__ out, int64_t n,
                                                     const uint64_t *__restrict__ offs) {
  __shared__ uint64_t lds[4];
  scan_chunk<uint64_t, uint64_t>(in, out, n, offs ? offs[blockIdx.x] : 0, lds);
}

// Exclusive scan of one chunk when the chunk sums are few (nb <= kFlatChunks):
// each block adds up the sums of the chunks before it itself, so no scan of
// the sums is launched.  Block 0 also writes the grand total (sums of chunks
// past the device count are 0) if `total` is given.
__global__ void __launch_bounds__(256) scan_down_flat_u32(const uint32_t *__restrict__ in,
                                                          uint32_t *__restrict__ out, int64_t n,
                                                          const uint64_t *__restrict__ n_dev,
                                                          const uint64_t *__restrict__ sums,
                                                          int64_t nb, uint64_t *__restrict__ total) {
  __shared__ uint64_t lds[4];
  n = eff_n(n, n_dev);
  if ((int64_t)blockIdx.x * kScanChunk >= n && !(blockIdx.x == 0 && total)) return;
  // block b: the sum of chunks 0 .. b-1; block 0 (offset 0): all nb chunks
  const int64_t upto = (blockIdx.x == 0 && total) ? nb : (int64_t)blockIdx.x;
  uint64_t acc = 0;
  for (int64_t j = threadIdx.x; j < upto; j += kBlock) acc += sums[j];
  uint64_t sum;
  block_exclusive_scan<uint64_t>(acc, lds, sum);
  if (blockIdx.x == 0 && total && threadIdx.x == 0) *total = sum;
  scan_chunk<uint32_t, uint32_t>(in, out, n, blockIdx.x == 0 ? 0 : sum, lds);
}

__global__ void scan_total(const uint64_t *__restrict__ excl, const uint64_t *__restrict__ sums,
                           int64_t nb, uint64_t *__restrict__ total) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *total = nb > 0 ? excl[nb - 1] + sums[nb - 1] : 0;
}

__global__ void single_total_u32(const uint32_t *__restrict__ in, int64_t n, uint64_t *total) {
  // only used for n <= one chunk
  __shared__ uint64_t lds[4];
  uint64_t acc = 0;
  for (int64_t i = threadIdx.x; i < n; i += kBlock) acc += in[i];
  uint64_t tot;
  block_exclusive_scan<uint64_t>(acc, lds, tot);
  if (threadIdx.x == 0) *total = tot;
}

int64_t nchunks(int64_t n) { return (n + kScanChunk - 1) / kScanChunk; }

// Exclusive scan of u64 values (recursive on chunk sums).
void scan_u64(const uint64_t *in, uint64_t *out, int64_t n, uint64_t *tmp, hipStream_t s) {
  const int64_t nb = nchunks(n);
  if (nb <= 1) {
    hipLaunchKernelGGL(scan_down_u64, dim3(1), dim3(kBlock), 0, s, in, out, n,
                       (const uint64_t *)nullptr);
    return;
  }
  uint64_t *sums = tmp, *offs = tmp + nb, *rest = tmp + 2 * nb;
  hipLaunchKernelGGL(scan_reduce_u64, dim3((unsigned)nb), dim3(kBlock), 0, s, in, n, sums);
  scan_u64(sums, offs, nb, rest, s);
  hipLaunchKernelGGL(scan_down_u64, dim3((unsigned)nb), dim3(kBlock), 0, s, in, out, n,
                     (const uint64_t *)offs);
}

size_t scan_u64_tmp(int64_t n) {
  const int64_t nb = nchunks(n);
  if (nb <= 1) return 0;
  return (size_t)(2 * nb) * sizeof(uint64_t) + scan_u64_tmp(nb);
}

// ----- gather and duplicate -----
__global__ void __launch_bounds__(256) gather_u32_kernel(const uint32_t *__restrict__ in,
                                                         const uint32_t *__restrict__ idx,
                                                         int64_t n,
                                                         const uint64_t *__restrict__ n_dev,
                                                         uint32_t *__restrict__ out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < eff_n(n, n_dev)) out[j] = in[idx[j]];
}

// One thread per instance in depth order: instance i = order[j] writes its
// pairs at offsets[j], in tile row-major order of its rectangle.
// key = global tile id, value = instance id i.
__device__ __forceinline__ void emit_pairs(const DevCam &c, int4 r, uint32_t i, uint64_t o,
                                           uint64_t cap, uint32_t *__restrict__ keys,
                                           uint32_t *__restrict__ vals,
                                           uint32_t *__restrict__ overflow) {
  const int tx0 = r.x >> 4, tx1 = r.z >> 4, ty0 = r.y >> 4, ty1 = r.w >> 4;
  for (int ty = ty0; ty <= ty1; ++ty)
    for (int tx = tx0; tx <= tx1; ++tx) {
      if (o < cap) {
        keys[o] = (uint32_t)(c.tile_base + ty * c.tiles_x + tx);
        vals[o] = i;
      } else if (overflow) {
        *overflow = 1u;
      }
      ++o;
    }
}

// Views of one scene: instance i = view * N + splat.
__global__ void __launch_bounds__(256)
duplicate_kernel(const uint32_t *__restrict__ order, const uint32_t *__restrict__ offsets,
                 const uint32_t *__restrict__ tiles, const int4 *__restrict__ rect,
                 const DevCam *__restrict__ cams, int64_t N, int64_t total,
                 uint32_t *__restrict__ keys, uint32_t *__restrict__ vals) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= total) return;
  const uint32_t i = order[j];
  if (tiles[i] == 0) return;
  emit_pairs(cams[i / N], rect[i], i, offsets[j], ~0ull, keys, vals, nullptr);
}

// A batch of slots; instance count on the device.  Pairs at or past `cap`
// are dropped and raise *overflow.
__global__ void __launch_bounds__(256)
duplicate_slots_kernel(const uint32_t *__restrict__ order, const uint32_t *__restrict__ offsets,
                       const uint32_t *__restrict__ tiles, const int4 *__restrict__ rect,
                       const Slot *__restrict__ slots, const int *__restrict__ n_slots,
                       int64_t inst_cap, const uint64_t *__restrict__ n_inst, uint64_t cap,
                       uint32_t *__restrict__ keys, uint32_t *__restrict__ vals,
                       uint32_t *__restrict__ overflow) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= eff_n(inst_cap, n_inst)) return;
  const uint32_t i = order[j];
  if (tiles[i] == 0) return;
  const Slot &sl = slots[slot_of_instance(slots, *n_slots, (int64_t)i)];
  emit_pairs(sl.cam, rect[i], i, offsets[j], cap, keys, vals, overflow);
}

// ----- radix sort -----
constexpr int kSortItems = 8;
// 2048 keys per chunk: the 1M-key depth sort then has 490 blocks, enough
// to fill the chip (123 us per depth sort at 1M keys, 132 with 4096).
constexpr int kSortChunk = kBlock * kSortItems;

__global__ void __launch_bounds__(256) radix_hist(const uint32_t *__restrict__ keys, int64_t n,
                                                  const uint64_t *__restrict__ n_dev, int shift,
                                                  int64_t nb, uint32_t *__restrict__ hist) {
  __shared__ uint32_t h[256];
  n = eff_n(n, n_dev);
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortChunk;
#pragma unroll
  for (int k = 0; k < kSortItems; ++k) {
    const int64_t i = base + (int64_t)k * kBlock + threadIdx.x;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter of one chunk of kSortChunk pairs: 1024 threads (16 wave64)
// rank the chunk in kSortChunk / 1024 rounds.  In a round each wave matches
// equal digits with 8 ballots; a per-digit prefix over the 16 waves (in
// wave order) and a running per-digit base carry the order across waves
// and rounds.
constexpr int kScatterThreads = 1024;
constexpr int kScatterWaves = kScatterThreads / 64;

__global__ void __launch_bounds__(kScatterThreads)
radix_scatter(const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin, int64_t n,
              const uint64_t *__restrict__ n_dev, int shift, int64_t nb,
              const uint32_t *__restrict__ offs, uint32_t *__restrict__ kout,
              uint32_t *__restrict__ vout) {
  __shared__ uint32_t base[256];                  // running count of each digit in this chunk
  __shared__ uint32_t wcnt[kScatterWaves][256];   // per-wave counts of the current round
  n = eff_n(n, n_dev);
  if ((int64_t)blockIdx.x * kSortChunk >= n) return;  // whole block past the end
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (tid < 256) base[tid] = offs[(int64_t)tid * nb + blockIdx.x];
  const int64_t chunk = (int64_t)blockIdx.x * kSortChunk;
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int k = 0; k < kSortChunk / kScatterThreads; ++k) {
    const int64_t i = chunk + (int64_t)k * kScatterThreads + tid;
    const bool ok = i < n;
    uint32_t key = 0, val = 0;
    if (ok) {
      key = kin[i];
      val = vin ? vin[i] : (uint32_t)i;  // no input values: value = index
    }
    const uint32_t d = (key >> shift) & 255u;
#pragma unroll
    for (int j = 0; j < kScatterWaves * 256 / kScatterThreads; ++j)
      (&wcnt[0][0])[j * kScatterThreads + tid] = 0;
    __syncthreads();
    // lanes of this wave with the same digit
    uint64_t peers = __ballot(ok);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint64_t m = __ballot((d >> b) & 1u);
      peers &= ((d >> b) & 1u) ? m : ~m;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & lt_mask);
    const uint32_t cnt = (uint32_t)__popcll(peers);
    const bool leader = ok && (peers >> lane) == 1ull;  // highest lane of its group
    if (leader) wcnt[w][d] = cnt;
    __syncthreads();
    // per digit: exclusive prefix over the waves in order
    if (tid < 256) {
      uint32_t b = base[tid];
#pragma unroll
      for (int v = 0; v < kScatterWaves; ++v) {
        const uint32_t c = wcnt[v][tid];
        wcnt[v][tid] = b;
        b += c;
      }
      base[tid] = b;
    }
    __syncthreads();
    if (ok) {
      const uint32_t pos = wcnt[w][d] + rank;
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
  }
}

__global__ void fill_u32_kernel(uint32_t *p, uint32_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void fill_f32_kernel(float *p, float v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// 16-byte stores for a 16-byte aligned array (n4 float4s).
__global__ void fill_f32x4_kernel(float4 *p, float v, int64_t n4) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n4) p[i] = make_float4(v, v, v, v);
}

__global__ void ranges_kernel(const uint32_t *__restrict__ keys, int64_t D,
                              const uint64_t *__restrict__ D_dev, uint2 *__restrict__ ranges) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  D = eff_n(D, D_dev);
  if (i >= D) return;
  const uint32_t t = keys[i];
  if (i == 0 || keys[i - 1] != t) ranges[t].x = (uint32_t)i;
  if (i == D - 1 || keys[i + 1] != t) ranges[t].y = (uint32_t)(i + 1);
}

}  // namespace

size_t scan_tmp_bytes(int64_t n) {
  const int64_t nb = nchunks(n);
  return (size_t)(2 * nb + 2) * sizeof(uint64_t) + scan_u64_tmp(nb);
}

void launch_scan(const uint32_t *in, uint32_t *out, int64_t n, uint64_t *total, void *tmp,
                 hipStream_t s, const uint64_t *n_dev) {
  if (n == 0) {
    hipLaunchKernelGGL(single_total_u32, dim3(1), dim3(kBlock), 0, s, in, (int64_t)0, total);
    return;
  }
  const int64_t nb = nchunks(n);
  uint64_t *sums = (uint64_t *)tmp, *offs = sums + nb, *rest = sums + 2 * nb + 2;
  hipLaunchKernelGGL(scan_reduce_u32, dim3((unsigned)nb), dim3(kBlock), 0, s, in, n, n_dev, sums);
  if (nb <= kFlatChunks) {
    hipLaunchKernelGGL(scan_down_flat_u32, dim3((unsigned)nb), dim3(kBlock), 0, s, in, out, n,
                       n_dev, (const uint64_t *)sums, nb, total);
    return;
  }
  scan_u64(sums, offs, nb, rest, s);
  hipLaunchKernelGGL(scan_down_u32, dim3((unsigned)nb), dim3(kBlock), 0, s, in, out, n, n_dev,
                     (const uint64_t *)offs);
  if (total)
    hipLaunchKernelGGL(scan_total, dim3(1), dim3(1), 0, s, (const uint64_t *)offs,
                       (const uint64_t *)sums, nb, total);
}

void launch_gather(const uint32_t *in, const uint32_t *idx, int64_t n, uint32_t *out,
                   hipStream_t s, const uint64_t *n_dev) {
  if (n <= 0) return;
  hipLaunchKernelGGL(gather_u32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in,
                     idx, n, n_dev, out);
}

void launch_duplicate(const uint32_t *order, const uint32_t *offsets, const uint32_t *tiles,
                      const int4 *rect, const DevCam *cams, int V, int64_t N, uint32_t *keys,
                      uint32_t *vals, hipStream_t s) {
  const int64_t total = (int64_t)V * N;
  if (total == 0) return;
  const int64_t nb = (total + 255) / 256;
  hipLaunchKernelGGL(duplicate_kernel, dim3((unsigned)nb), dim3(256), 0, s, order, offsets, tiles,
                     rect, cams, N, total, keys, vals);
}

void launch_duplicate_slots(const uint32_t *order, const uint32_t *offsets,
                            const uint32_t *tiles, const int4 *rect, const Slot *slots,
                            const int *n_slots, int64_t inst_cap, const uint64_t *n_inst,
                            uint64_t pair_cap, uint32_t *keys, uint32_t *vals,
                            uint32_t *overflow, hipStream_t s) {
  if (inst_cap <= 0) return;
  hipLaunchKernelGGL(duplicate_slots_kernel, dim3((unsigned)((inst_cap + 255) / 256)), dim3(256),
                     0, s, order, offsets, tiles, rect, slots, n_slots, inst_cap, n_inst, pair_cap,
                     keys, vals, overflow);
}

size_t sort_tmp_bytes(int64_t n) {
  const int64_t nb = (n + kSortChunk - 1) / kSortChunk;
  const int64_t h = 256 * std::max<int64_t>(nb, 1);
  return (size_t)(2 * h) * sizeof(uint32_t) + scan_tmp_bytes(h) + 64;
}

int launch_radix_sort(const uint32_t *k0, const uint32_t *v0, uint32_t *ka, uint32_t *va,
                      uint32_t *kb, uint32_t *vb, int64_t n, int bits, void *tmp, hipStream_t s,
                      const uint64_t *n_dev) {
  if (n <= 0) return 0;
  const int64_t nb = (n + kSortChunk - 1) / kSortChunk;
  const int64_t h = 256 * nb;
  uint32_t *hist = (uint32_t *)tmp;
  uint32_t *offs = hist + h;
  uint64_t *total = (uint64_t *)(offs + h);
  void *stmp = (void *)(total + 1);
  const uint32_t *kin = k0, *vin = v0;
  uint32_t *kout = ka, *vout = va;
  int which = 0;
  const int passes = bits <= 8 ? 1 : (bits + 7) / 8;
  for (int p = 0; p < passes; ++p) {
    const int shift = 8 * p;
    hipLaunchKernelGGL(radix_hist, dim3((unsigned)nb), dim3(kBlock), 0, s, kin, n, n_dev, shift,
                       nb, hist);
    launch_scan(hist, offs, h, nullptr, stmp, s);
    hipLaunchKernelGGL(radix_scatter, dim3((unsigned)nb), dim3(kScatterThreads), 0, s, kin, vin, n,
                       n_dev, shift, nb, (const uint32_t *)offs, kout, vout);
    which = (kout == ka) ? 0 : 1;
    kin = kout;
    vin = vout;
    kout = (which == 0) ? kb : ka;
    vout = (which == 0) ? vb : va;
  }
  return which;
}

void launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, v, n);
}

void launch_fill_f32(float *p, float v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  if ((reinterpret_cast<uintptr_t>(p) & 15u) == 0 && n >= 4) {
    const int64_t n4 = n / 4, tail = n - 4 * n4;
    hipLaunchKernelGGL(fill_f32x4_kernel, dim3((unsigned)((n4 + 255) / 256)), dim3(256), 0, s,
                       reinterpret_cast<float4 *>(p), v, n4);
    if (tail)
      hipLaunchKernelGGL(fill_f32_kernel, dim3(1), dim3(256), 0, s, p + 4 * n4, v, tail);
    return;
  }
  hipLaunchKernelGGL(fill_f32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, v, n);
}

void launch_ranges(const uint32_t *keys, int64_t D, uint2 *ranges, hipStream_t s,
                   const uint64_t *D_dev) {
  if (D <= 0) return;
  hipLaunchKernelGGL(ranges_kernel, dim3((unsigned)((D + 255) / 256)), dim3(256), 0, s, keys, D,
                     D_dev, ranges);
}

}  // namespace hgs
