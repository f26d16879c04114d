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
// The radix sort uses 8-bit digits: one up-front launch counts the digits
// of every pass, and each pass is a single launch that ranks 8192- or
// 4096-key chunks (16 wave64 per chunk, wave ballots for equal digits) and finds
// each chunk's place by a decoupled look-back over the chunks before it.

#include "hgs_internal.h"

namespace hgs {

namespace {

constexpr int kScanItems = 16;                       // elements per thread
constexpr int kScanChunk = kBlock * kScanItems;      // 4096 per block
constexpr int64_t kFlatChunks = 4096;  // up to 16M elements: two launches per scan

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

// Pairs of the wave of 64 consecutive entries j0 .. j0 + 63 (below
// `total`) of the depth order.  Their runs [offsets[j], offsets[j] + count)
// are contiguous, and the lanes write the wave's pairs 64 at a time, each
// lane finding the entry that owns its position by a binary search over the
// lanes' run starts: the stores are coalesced, and a splat with many tiles
// does not hold up the other 63 lanes.  The tile rectangles come packed and
// in depth order (prect_s[j]), so the reads are sequential; an instance
// whose rectangle does not fit the packed form (kWideRect) reads tiles[i]
// and rect[i].  cam_of(i) gives an instance's camera.  Pairs at or past
// `cap` are dropped and raise *overflow.
template <class CamOf>
__device__ __forceinline__ void duplicate_wave(int64_t j0, int64_t total,
                                               const uint32_t *__restrict__ order,
                                               const uint32_t *__restrict__ offsets,
                                               const uint32_t *__restrict__ tiles,
                                               const int4 *__restrict__ rect,
                                               const uint32_t *__restrict__ prect_s,
                                               CamOf cam_of, uint64_t cap,
                                               uint32_t *__restrict__ keys,
                                               uint32_t *__restrict__ vals,
                                               uint32_t *__restrict__ overflow) {
  const int lane = threadIdx.x & 63;
  const int64_t j = j0 + lane;
  const bool in = j < total;
  const uint64_t vm = __ballot(in);
  if (vm == 0ull) return;  // in-range lanes are a prefix of the wave
  uint32_t i = 0, cnt = 0, o = 0;
  int tx0 = 0, ty0 = 0, w = 1;
  if (in) {
    i = order[j];
    o = offsets[j];
    const uint32_t pr = prect_s[j];
    if (pr == kWideRect) {
      cnt = tiles[i];
      const int4 r = rect[i];
      tx0 = r.x >> 4;
      ty0 = r.y >> 4;
      w = (r.z >> 4) - tx0 + 1;
    } else {
      cnt = packed_tile_count(pr);
      tx0 = (int)(pr & 255u);
      ty0 = (int)((pr >> 8) & 255u);
      w = (int)((pr >> 16) & 255u) + 1;
    }
  }
  const uint32_t o0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)o);
  // run start relative to the wave's first pair (out of range: never owns)
  const uint32_t st = in ? o - o0 : 0xffffffffu;
  const int last = 63 - __builtin_clzll(vm);
  const uint32_t T = (uint32_t)__builtin_amdgcn_readlane((int)(st + cnt), last);
  // key of the run's q-th pair: base + (q / w) tiles_x + q % w
  int base = 0, txs = 1;
  if (in && cnt) {
    const DevCam &c = cam_of(i);
    txs = c.tiles_x;
    base = c.tile_base + ty0 * c.tiles_x + tx0;
  }
  for (uint32_t p = (uint32_t)lane; p < T + 63u - (T + 63u) % 64u; p += 64u) {
    // the last lane k with st_k <= p (a zero-length run shares its start with
    // the next lane's, so the owner has pairs)
    int k = 0;
#pragma unroll
    for (int step = 32; step >= 1; step >>= 1) {
      const uint32_t sc = (uint32_t)__shfl((int)st, k + step);
      k = sc <= p ? k + step : k;
    }
    const uint32_t sk = (uint32_t)__shfl((int)st, k);
    const int bk = __shfl(base, k), xk = __shfl(txs, k), wk = __shfl(w, k);
    const uint32_t ik = (uint32_t)__shfl((int)i, k);
    if (p >= T) continue;
    const uint32_t q = p - sk;
    // q / wk by a reciprocal, corrected to the exact quotient
    uint32_t row = (uint32_t)((float)q * __builtin_amdgcn_rcpf((float)wk));
    row -= row * (uint32_t)wk > q ? 1u : 0u;
    row += (row + 1u) * (uint32_t)wk <= q ? 1u : 0u;
    const uint32_t col = q - row * (uint32_t)wk;
    const uint64_t pos = (uint64_t)o0 + p;
    if (pos < cap) {
      keys[pos] = (uint32_t)(bk + (int)row * xk + (int)col);
      vals[pos] = ik;
    } else if (overflow) {
      *overflow = 1u;
    }
  }
}

// Views of one scene: instance i = view * N + splat, one wave per 64
// entries.  zero[0, zero_n) is cleared by the same launch.
__global__ void __launch_bounds__(256)
duplicate_kernel(const uint32_t *__restrict__ order, const uint32_t *__restrict__ offsets,
                 const uint32_t *__restrict__ tiles, const int4 *__restrict__ rect,
                 const uint32_t *__restrict__ prect_s, const DevCam *__restrict__ cams,
                 int64_t N, int64_t total, uint64_t cap, uint32_t *__restrict__ keys,
                 uint32_t *__restrict__ vals, uint32_t *__restrict__ overflow,
                 uint32_t *__restrict__ zero, int64_t zero_n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t z = t; z < zero_n; z += (int64_t)gridDim.x * blockDim.x) zero[z] = 0u;
  duplicate_wave(t & ~int64_t(63), total, order, offsets, tiles, rect, prect_s,
                 [&](uint32_t i) -> const DevCam & { return cams[i / N]; }, cap, keys, vals,
                 overflow);
}

struct CamPack {
  DevCam c[kCamsPerUpload];
};

__global__ void upload_cams_kernel(CamPack p, int n, DevCam *__restrict__ dst, ZeroList z) {
  // 8-byte words of n cameras (DevCam is 8-byte aligned)
  constexpr int kWords = (int)(sizeof(DevCam) / 8);
  static_assert(sizeof(DevCam) % 8 == 0, "DevCam is copied in 8-byte words");
  for (int k = threadIdx.x; k < n * kWords; k += blockDim.x)
    reinterpret_cast<uint2 *>(dst)[k] = reinterpret_cast<const uint2 *>(p.c)[k];
  // small arrays the render needs cleared (counters, flags), in the same launch
#pragma unroll
  for (int a = 0; a < ZeroList::kMax; ++a)
    for (int k = threadIdx.x; k < z.n[a]; k += blockDim.x) z.p[a][k] = 0u;
}

// A batch of slots; instance count on the device (the grid strides over
// waves of 64 entries).  Pairs at or past `cap` are dropped and raise
// *overflow.
__global__ void __launch_bounds__(256)
duplicate_slots_kernel(const uint32_t *__restrict__ order, const uint32_t *__restrict__ offsets,
                       const uint32_t *__restrict__ tiles, const int4 *__restrict__ rect,
                       const uint32_t *__restrict__ prect_s, const Slot *__restrict__ slots,
                       const int *__restrict__ n_slots, int64_t inst_cap,
                       const uint64_t *__restrict__ n_inst, uint64_t cap,
                       uint32_t *__restrict__ keys, uint32_t *__restrict__ vals,
                       uint32_t *__restrict__ overflow) {
  const int64_t cnt = eff_n(inst_cap, n_inst);
  const int ns = *n_slots;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) & ~int64_t(63); j0 < cnt;
       j0 += stride)
    duplicate_wave(j0, cnt, order, offsets, tiles, rect, prect_s,
                   [&](uint32_t i) -> const DevCam & {
                     return slots[slot_of_instance(slots, ns, (int64_t)i)].cam;
                   },
                   cap, keys, vals, overflow);
}

// ----- radix sort: one sweep per digit -----
//
// An up-front kernel counts the digits of every pass at once (the global
// digit totals of a pass do not depend on the order the earlier passes
// leave).  Each pass is then one kernel over chunks of 8192 (or 4096) keys.  A
// chunk takes a ticket from an atomic counter (tickets follow the order in
// which blocks start, so a chunk only ever waits for chunks that are
// already running), ranks its keys in input order, publishes its per-digit
// counts, and looks back over the earlier chunks' published counts (each a
// 64-bit word: 2 flag bits, aggregate or inclusive prefix, and the value)
// until it meets an inclusive prefix.  Its keys then go to
//   global digit offset + prefix of earlier chunks + rank within the chunk.
// A pass whose digit is the same for every key is the identity and only
// copies.  Status tables alternate between passes; each chunk clears its
// row of the other table for the next pass, and the up-front kernel clears
// the first pass's table.  A look-back that does not complete within a
// bounded number of waits sets bit 1 of *err and gives up (the order is
// then wrong but every wave ends).
constexpr int kOsThreads = 1024;
constexpr int kOsWaves = kOsThreads / 64;
// Keys per thread: 8 (8192-key chunks), or 4 (4096-key chunks) for a sort
// whose small-chunk count still fits one resident block per CU
// (kSmallChunkCap): a pass costs about one chunk's latency per round of
// resident chunks, so more, shorter chunks finish sooner there.
constexpr int kOsRowsBig = 8, kOsRowsSmall = 4;
constexpr int64_t kSmallChunkCap = 256;
constexpr int kPartWin = 12;  // look-back words per thread per round (4 parts: 48 per digit)
constexpr int kMaxPasses = 4;
constexpr int kOsWords = kSortWords;  // hist [pass][256], tickets [pass], zero keys
constexpr int kZeroWord = kMaxPasses * 256 + kMaxPasses;  // count of keys equal to 0
static_assert(kSortWords == kMaxPasses * 256 + kMaxPasses + 1, "sort words layout");
constexpr size_t kOsHead = 4352;                  // bytes before the status tables
constexpr uint64_t kFlagAgg = 1ull << 62, kFlagInc = 2ull << 62;
constexpr uint64_t kValMask = (1ull << 62) - 1;
constexpr int kSpinLimit = 1 << 16;  // look-back rounds before giving up
constexpr int kOsMaxBlocks = 1024;  // persistent grid of a pass (two per CU and more)



// Digit counts of all passes (atomics into hist[pass][256], zeroed before),
// and the first pass's status table cleared.  Each thread counts groups of 8
// consecutive keys and adds runs of equal digits with one LDS atomic: the
// pairs of one splat are adjacent and share their depth digits, so most runs
// are long.  kVec: keys is 16-byte aligned (two 16-byte loads per group).
constexpr int kHistThreads = 1024;
constexpr int kHistMaxBlocks = 512;
template <bool kVec>
__global__ void __launch_bounds__(kHistThreads)
radix_hist_all(const uint32_t *__restrict__ keys, int64_t n, const uint64_t *__restrict__ n_dev,
               int passes, int chunk, uint32_t *__restrict__ hist,
               uint64_t *__restrict__ st0) {
  __shared__ uint32_t h[kMaxPasses][256];
  __shared__ uint32_t s_zero;  // keys equal to 0
  n = eff_n(n, n_dev);
  for (int k = threadIdx.x; k < kMaxPasses * 256; k += kHistThreads) (&h[0][0])[k] = 0;
  if (threadIdx.x == 0) s_zero = 0;
  __syncthreads();
  uint32_t zeros = 0;
  const int64_t stride = (int64_t)gridDim.x * kHistThreads;
  const int64_t groups = (n + 7) >> 3;
  for (int64_t g = (int64_t)blockIdx.x * kHistThreads + threadIdx.x; g < groups; g += stride) {
    const int64_t i0 = g << 3;
    const int m = n - i0 < 8 ? (int)(n - i0) : 8;
    uint32_t k[8];
    if (kVec && m == 8) {
      const uint4 a = reinterpret_cast<const uint4 *>(keys)[2 * g];
      const uint4 b = reinterpret_cast<const uint4 *>(keys)[2 * g + 1];
      k[0] = a.x; k[1] = a.y; k[2] = a.z; k[3] = a.w;
      k[4] = b.x; k[5] = b.y; k[6] = b.z; k[7] = b.w;
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) k[j] = j < m ? keys[i0 + j] : 0u;
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) zeros += (j < m && k[j] == 0u) ? 1u : 0u;
    for (int p = 0; p < passes; ++p) {
      const int sh = 8 * p;
      uint32_t d = (k[0] >> sh) & 255u, c = 1;
#pragma unroll
      for (int j = 1; j < 8; ++j) {
        if (j < m) {
          const uint32_t e = (k[j] >> sh) & 255u;
          if (e != d) {
            atomicAdd(&h[p][d], c);
            d = e;
            c = 0;
          }
          ++c;
        }
      }
      atomicAdd(&h[p][d], c);
    }
  }
  const int64_t rows = (n + chunk - 1) / chunk * 256;
  for (int64_t i = (int64_t)blockIdx.x * kHistThreads + threadIdx.x; i < rows; i += stride)
    st0[i] = 0;
  if (zeros) atomicAdd(&s_zero, zeros);
  __syncthreads();
  for (int k = threadIdx.x; k < passes * 256; k += kHistThreads) {
    const uint32_t c = (&h[0][0])[k];
    if (c) atomicAdd(&hist[k], c);
  }
  if (threadIdx.x == 0 && s_zero) atomicAdd(&hist[kZeroWord], s_zero);
}

__device__ __forceinline__ void gather_put(const uint32_t *__restrict__ gsrc,
                                           const uint32_t *__restrict__ gtiles,
                                           uint32_t *__restrict__ gdst,
                                           uint32_t *__restrict__ gdst2, uint32_t v,
                                           int64_t pos) {
  const uint32_t x = gsrc[v];
  if (gdst2) {
    gdst[pos] = x == kWideRect ? gtiles[v] : packed_tile_count(x);
    gdst2[pos] = x;
  } else {
    gdst[pos] = x;
  }
}

// The buffers of one sort.  k0/v0 the input (v0 NULL: the values are the
// keys' input indices), (ka, va) and (kb, vb) the ping-pong pair, st[2] the
// status tables.  skip: passes whose digit is the same for every key are
// skipped on the device (k0 must then alias neither ka nor kb); with
// zero_free, for every key other than 0 (keys equal to 0 then keep their
// relative order but not their place among the others).
struct SortIO {
  const uint32_t *k0, *v0;
  uint32_t *kbuf[2], *vbuf[2];
  uint64_t *st[2];
  int passes;
  int skip;
  int zero_free;  // keys equal to 0 are don't-care: they may end anywhere
};

// One pass, on a persistent grid: each block takes chunk tickets until they
// run out.  Its input, output and status tables follow from the passes that
// do work: without skipping, pass p reads the input (p = 0) or buffer
// (p - 1) & 1 and writes buffer p & 1.  With skipping, a pass whose digit is
// constant (all the keys in one bucket of the up-front histogram) exits at
// once, and the k-th of the M passes that remain writes buffer
// E ^ ((M - 1 - k) & 1), E = (passes - 1) & 1, so the last one leaves the
// result where the host expects it; if every pass is constant the last one
// copies the input there.  Only the pass that writes the result does the
// gather: gsrc/gdst (may be NULL) write gdst[pos] = gsrc[value]; with
// gdst2, gsrc holds packed tile rectangles: gdst[pos] = their tile counts
// (from gtiles for a kWideRect word) and gdst2[pos] = the words.
template <int kRows>
__global__ void __launch_bounds__(kOsThreads)
radix_onesweep(SortIO io, int64_t n, const uint64_t *__restrict__ n_dev, int pass,
               uint32_t *__restrict__ words, const uint32_t *__restrict__ gsrc_in,
               const uint32_t *__restrict__ gtiles, uint32_t *__restrict__ gdst_in,
               uint32_t *__restrict__ gdst2, uint32_t *__restrict__ err) {
  __shared__ uint32_t s_whist[kOsWaves][256];  // per-wave digit counts, then offsets
  __shared__ uint32_t s_gex[256];              // global exclusive digit offsets
  __shared__ uint32_t s_base[256];             // + the earlier chunks of this one
  __shared__ uint32_t s_wtot[4];
  __shared__ uint32_t s_ticket;
  __shared__ int s_trivial;
  __shared__ uint32_t s_run[256];         // this chunk's digit counts
  __shared__ int64_t s_lj[256];           // look-back position per digit
  __shared__ uint64_t s_lex[256];         // prefix gathered so far per digit
  __shared__ int s_ldone[256];
  __shared__ uint4 s_lpart[4][256];       // a round's part results
  __shared__ int s_lany;
  __shared__ uint32_t s_cex[256];         // chunk-local exclusive digit offsets
  constexpr int kChunk = kOsThreads * kRows;
  __shared__ uint32_t s_key[kChunk];      // the chunk in digit order
  __shared__ uint32_t s_val[kChunk];
  __shared__ uint32_t s_const;             // bit q: pass q's digit is constant
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int shift = 8 * pass;
  n = eff_n(n, n_dev);
  const int64_t nch = (n + kChunk - 1) / kChunk;
  if ((int64_t)blockIdx.x >= nch) return;  // more blocks than chunks
  if (tid == 0) {
    s_trivial = 0;
    s_const = 0;
  }
  __syncthreads();
  if (tid < 256) {
    const int64_t nz = io.zero_free ? (int64_t)words[kZeroWord] : 0;
    for (int q = 0; q < io.passes; ++q) {
      const int64_t c = (int64_t)words[q * 256 + tid] - (tid == 0 ? nz : 0);
      if (c == n - nz) atomicOr(&s_const, 1u << q);
    }
  }
  __syncthreads();
  // this pass's place among the passes that do work
  const uint32_t cmask = s_const;
  const uint32_t all = (1u << io.passes) - 1u;
  const int M = io.skip ? io.passes - __popc(cmask & all) : io.passes;
  const int k = io.skip ? pass - __popc(cmask & ((1u << pass) - 1u)) : pass;
  const bool mine_const = (cmask >> pass) & 1u;
  const bool copy_all = io.skip && M == 0 && pass == io.passes - 1;
  if (io.skip && mine_const && !copy_all) return;  // block-uniform
  const int E = (io.passes - 1) & 1;
  const int ob = io.skip ? (copy_all ? E : (E ^ ((M - 1 - k) & 1))) : (pass & 1);
  const bool first = copy_all || k == 0;
  const bool last = copy_all || k == M - 1;
  const uint32_t *__restrict__ kin = first ? io.k0 : io.kbuf[ob ^ 1];
  const uint32_t *__restrict__ vin = first ? io.v0 : io.vbuf[ob ^ 1];
  uint32_t *__restrict__ kout = io.kbuf[ob];
  uint32_t *__restrict__ vout = io.vbuf[ob];
  const int sk = copy_all ? 0 : k;
  uint64_t *__restrict__ st_cur = io.st[sk & 1];
  uint64_t *__restrict__ st_next = io.st[(sk + 1) & 1];
  const bool gen_idx = vin == nullptr;  // first pass over index values
  const uint32_t *__restrict__ gsrc = last ? gsrc_in : nullptr;
  uint32_t *__restrict__ gdst = last ? gdst_in : nullptr;
  // global exclusive digit offsets of this pass
  uint32_t g = 0, gx = 0;
  if (tid < 256) {
    g = words[pass * 256 + tid];
    gx = g;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t y = __shfl_up(gx, d, 64);
      if (lane >= d) gx += y;
    }
    if (lane == 63) s_wtot[w] = gx;
  }
  __syncthreads();
  if (tid < 256) {
    uint32_t off = 0;
    for (int k = 0; k < w; ++k) off += s_wtot[k];
    s_gex[tid] = off + gx - g;
    if ((int64_t)g == n || copy_all) s_trivial = 1;
  }
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

  for (;;) {
    if (tid == 0) s_ticket = atomicAdd(&words[kMaxPasses * 256 + pass], 1u);
    for (int k = tid; k < kOsWaves * 256; k += kOsThreads) (&s_whist[0][0])[k] = 0;
    __syncthreads();
    const int64_t chunk = (int64_t)s_ticket;
    if (chunk >= nch) return;  // block-uniform
    if (tid < 256) st_next[chunk * 256 + tid] = 0;  // the next pass's row
    const int64_t c0 = chunk * kChunk;

    if (s_trivial) {  // one digit for all keys: the identity
#pragma unroll
      for (int j = 0; j < kRows; ++j) {
        const int64_t i = c0 + (int64_t)j * kOsThreads + tid;
        if (i < n) {
          const uint32_t v = gen_idx ? (uint32_t)i : vin[i];
          kout[i] = kin[i];
          vout[i] = v;
          if (gdst) gather_put(gsrc, gtiles, gdst, gdst2, v, i);
        }
      }
      __syncthreads();  // s_ticket is read before the next ticket overwrites it
      continue;
    }

    // each wave owns 64 kRows consecutive keys, as kRows rows of 64
    const int64_t wb = c0 + (int64_t)w * (64 * kRows);
    uint32_t key[kRows], val[kRows], rank[kRows];
    bool ok[kRows];
#pragma unroll
    for (int j = 0; j < kRows; ++j) {
      const int64_t i = wb + (int64_t)j * 64 + lane;
      ok[j] = i < n;
      key[j] = ok[j] ? kin[i] : 0u;
      val[j] = ok[j] ? (gen_idx ? (uint32_t)i : vin[i]) : 0u;
    }
#pragma unroll
    for (int j = 0; j < kRows; ++j) {
      const uint32_t d = (key[j] >> shift) & 255u;
      uint64_t peers = __ballot(ok[j]);
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const uint64_t m = __ballot((d >> b) & 1u);
        peers &= ((d >> b) & 1u) ? m : ~m;
      }
      const uint32_t prev = ok[j] ? s_whist[w][d] : 0u;
      rank[j] = prev + (uint32_t)__popcll(peers & lt_mask);
      // the highest lane of each group advances the wave's count; the reads
      // above are issued by the whole wave before this write
      if (ok[j] && (peers >> lane) == 1ull) s_whist[w][d] = prev + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    if (tid < 256) {
      uint32_t run = 0;
#pragma unroll
      for (int v = 0; v < kOsWaves; ++v) {
        const uint32_t c = s_whist[v][tid];
        s_whist[v][tid] = run;
        run += c;
      }
      s_run[tid] = run;
      uint64_t *me = st_cur + chunk * 256 + tid;
      __hip_atomic_store(me, (chunk == 0 ? kFlagInc : kFlagAgg) | (uint64_t)run, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
      s_lj[tid] = chunk - 1;
      s_lex[tid] = 0;
      s_ldone[tid] = chunk == 0 ? 1 : 0;
    }
    __syncthreads();
    // Look-back, all 16 waves: digit d = tid % 256 is read by four parts
    // p = tid / 256, each reading kPartWin words of the 4 kPartWin words
    // before the digit's current position; the parts are combined in order.
    for (int spins = 0;; ++spins) {
      if (s_lany == 0 && spins > 0) break;
      const int d = tid & 255, part = tid >> 8;
      if (!s_ldone[d]) {
        const int64_t j0 = s_lj[d] - (int64_t)part * kPartWin;
        uint64_t v[kPartWin];
#pragma unroll
        for (int k = 0; k < kPartWin; ++k) {
          const int64_t jj = j0 - k < 0 ? 0 : j0 - k;
          v[k] = __hip_atomic_load(st_cur + jj * 256 + d, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
        uint64_t sum = 0;
        uint32_t cnt = 0, state = 0;  // 0 all aggregates, 1 inclusive found, 2 stalled
#pragma unroll
        for (int k = 0; k < kPartWin; ++k) {
          if (state != 0) continue;
          const uint64_t f = v[k] & ~kValMask;
          if (f == 0) {
            state = 2;
            continue;
          }
          sum += v[k] & kValMask;
          ++cnt;
          if (f == kFlagInc) state = 1;
        }
        s_lpart[part][d] = make_uint4((uint32_t)sum, (uint32_t)(sum >> 32), cnt, state);
      }
      __syncthreads();
      if (tid == 0) s_lany = 0;
      __syncthreads();
      if (tid < 256 && !s_ldone[tid]) {
        uint64_t ex = s_lex[tid];
        int64_t j = s_lj[tid];
        bool done = false, stall = false;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (done || stall) continue;
          const uint4 r = s_lpart[q][tid];
          ex += (uint64_t)r.x | ((uint64_t)r.y << 32);
          j -= r.z;
          done = r.w == 1;
          stall = r.w == 2;
        }
        if (!done && spins > kSpinLimit) {
          if (err) atomicOr(err, 2u);
          done = true;
        }
        s_lex[tid] = ex;
        s_lj[tid] = j;
        s_ldone[tid] = done ? 1 : 0;
        if (!done) {
          s_lany = 1;
          if (stall) __builtin_amdgcn_s_sleep(1);
        }
      }
      __syncthreads();
    }
    // chunk-local exclusive offsets of the digits
    uint32_t r = 0, rx = 0;
    if (tid < 256) {
      const uint64_t excl = s_lex[tid];
      r = s_run[tid];
      if (chunk > 0)
        __hip_atomic_store(st_cur + chunk * 256 + tid, kFlagInc | (excl + r), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
      s_base[tid] = s_gex[tid] + (uint32_t)excl;
      rx = r;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(rx, d, 64);
        if (lane >= d) rx += y;
      }
      if (lane == 63) s_wtot[w] = rx;
    }
    __syncthreads();
    if (tid < 256) {
      uint32_t off = 0;
      for (int k = 0; k < w; ++k) off += s_wtot[k];
      s_cex[tid] = off + rx - r;
    }
    __syncthreads();
    // the chunk sorted by digit in LDS, so that each digit's run is written
    // out by consecutive threads (coalesced) rather than key by key
#pragma unroll
    for (int j = 0; j < kRows; ++j) {
      if (!ok[j]) continue;
      const uint32_t d = (key[j] >> shift) & 255u;
      const uint32_t lp = s_cex[d] + s_whist[w][d] + rank[j];
      s_key[lp] = key[j];
      s_val[lp] = val[j];
    }
    __syncthreads();
    const int cn = (int)(n - c0 < kChunk ? n - c0 : kChunk);
#pragma unroll
    for (int j = 0; j < kRows; ++j) {
      const int e = j * kOsThreads + tid;
      if (e >= cn) continue;
      const uint32_t k = s_key[e], v = s_val[e];
      const uint32_t d = (k >> shift) & 255u;
      const uint32_t pos = s_base[d] + (uint32_t)e - s_cex[d];
      kout[pos] = k;
      vout[pos] = v;
      if (gdst) gather_put(gsrc, gtiles, gdst, gdst2, v, pos);
    }
    __syncthreads();  // LDS is read before the next chunk clears it
  }
}

__global__ void fill_u32_kernel(uint32_t *p, uint32_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Every region of f set to zero: a grid-stride loop over their concatenation.
__global__ void zero_list_kernel(FillList f, int64_t total) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
    int64_t k = i;
#pragma unroll
    for (int a = 0; a < FillList::kMax; ++a) {
      if (k >= 0 && k < f.n[a]) f.p[a][k] = 0u;
      k -= f.n[a];
    }
  }
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
  D = eff_n(D, D_dev);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < D;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t t = keys[i];
    if (i == 0 || keys[i - 1] != t) ranges[t].x = (uint32_t)i;
    if (i == D - 1 || keys[i + 1] != t) ranges[t].y = (uint32_t)(i + 1);
  }
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
                      const int4 *rect, const uint32_t *prect_sorted, const DevCam *cams, int V,
                      int64_t N, uint64_t pair_cap, uint32_t *keys, uint32_t *vals,
                      uint32_t *overflow, uint32_t *zero, int64_t zero_n, hipStream_t s) {
  const int64_t total = (int64_t)V * N;
  if (total == 0) {
    if (zero_n > 0) launch_fill_u32(zero, 0u, zero_n, s);
    return;
  }
  const int64_t nb = (total + 255) / 256;
  hipLaunchKernelGGL(duplicate_kernel, dim3((unsigned)nb), dim3(256), 0, s, order, offsets, tiles,
                     rect, prect_sorted, cams, N, total, pair_cap, keys, vals, overflow, zero,
                     zero_n);
}

void launch_upload_cams(const DevCam *host, int n, DevCam *dst, hipStream_t s, ZeroList z) {
  for (int b = 0; b < n; b += kCamsPerUpload) {
    CamPack p;
    const int m = n - b < kCamsPerUpload ? n - b : kCamsPerUpload;
    for (int k = 0; k < m; ++k) p.c[k] = host[b + k];
    hipLaunchKernelGGL(upload_cams_kernel, dim3(1), dim3(256), 0, s, p, m, dst + b,
                       b == 0 ? z : ZeroList{});
  }
}

void launch_duplicate_slots(const uint32_t *order, const uint32_t *offsets,
                            const uint32_t *tiles, const int4 *rect, const uint32_t *prect_sorted,
                            const Slot *slots, const int *n_slots, int64_t inst_cap,
                            const uint64_t *n_inst, uint64_t pair_cap, uint32_t *keys,
                            uint32_t *vals, uint32_t *overflow, hipStream_t s) {
  if (inst_cap <= 0) return;
  const int64_t blocks = std::min<int64_t>((inst_cap + 255) / 256, 4096);
  hipLaunchKernelGGL(duplicate_slots_kernel, dim3((unsigned)blocks), dim3(256), 0, s, order,
                     offsets, tiles, rect, prect_sorted, slots, n_slots, inst_cap, n_inst,
                     pair_cap, keys, vals, overflow);
}

// chunk size of a sort of n keys (capacity n)
static int sort_rows(int64_t n) {
  const int64_t small = kOsThreads * kOsRowsSmall;
  return (n + small - 1) / small <= kSmallChunkCap ? kOsRowsSmall : kOsRowsBig;
}

// Enough for a sort of any m <= n keys (either chunk size).
size_t sort_tmp_bytes(int64_t n) {
  const int64_t big = (int64_t)kOsThreads * kOsRowsBig, small = (int64_t)kOsThreads * kOsRowsSmall;
  const int64_t nch = std::max<int64_t>(
      std::max<int64_t>((n + big - 1) / big, std::min<int64_t>((n + small - 1) / small,
                                                               kSmallChunkCap)),
      1);
  return kOsHead + (size_t)(2 * nch * 256) * sizeof(uint64_t);
}



int launch_radix_sort(const uint32_t *k0, const uint32_t *v0, uint32_t *ka, uint32_t *va,
                      uint32_t *kb, uint32_t *vb, int64_t n, int bits, void *tmp, hipStream_t s,
                      const uint64_t *n_dev, const uint32_t *gather_src, uint32_t *gather_dst,
                      uint32_t *err, uint32_t *zeroed_words, uint32_t *gather_dst2,
                      const uint32_t *gather_tiles, bool zero_free) {
  if (n <= 0) return 0;
  const int rows = sort_rows(n);
  const int chunk = kOsThreads * rows;
  const int64_t nch = (n + chunk - 1) / chunk;
  uint32_t *words = zeroed_words ? zeroed_words : (uint32_t *)tmp;
  uint64_t *st[2] = {(uint64_t *)((char *)tmp + kOsHead),
                     (uint64_t *)((char *)tmp + kOsHead) + nch * 256};
  const int passes = bits <= 8 ? 1 : (bits + 7) / 8;
  if (!zeroed_words) launch_fill_u32(words, 0u, kOsWords, s);
  // two blocks per CU at most: each adds its histograms to the global table
  // with atomics on the same passes x 256 addresses as every other block
  const int64_t hb =
      std::min<int64_t>((n + 8 * kHistThreads - 1) / (8 * kHistThreads), kHistMaxBlocks);
  if (((uintptr_t)k0 & 15) == 0)
    hipLaunchKernelGGL(radix_hist_all<true>, dim3((unsigned)hb), dim3(kHistThreads), 0, s, k0,
                       n, n_dev, passes, chunk, words, st[0]);
  else
    hipLaunchKernelGGL(radix_hist_all<false>, dim3((unsigned)hb), dim3(kHistThreads), 0, s, k0,
                       n, n_dev, passes, chunk, words, st[0]);
  SortIO io;
  io.k0 = k0;
  io.v0 = v0;
  io.kbuf[0] = ka;
  io.vbuf[0] = va;
  io.kbuf[1] = kb;
  io.vbuf[1] = vb;
  io.st[0] = st[0];
  io.st[1] = st[1];
  io.passes = passes;
  // a constant-digit pass can be skipped only if the input stays intact
  io.skip = (k0 != ka && k0 != kb && (v0 == nullptr || (v0 != va && v0 != vb))) ? 1 : 0;
  io.zero_free = io.skip && zero_free ? 1 : 0;
  const unsigned grid = (unsigned)std::min<int64_t>(nch, kOsMaxBlocks);
  for (int p = 0; p < passes; ++p) {
    if (rows == kOsRowsSmall)
      hipLaunchKernelGGL(radix_onesweep<kOsRowsSmall>, dim3(grid), dim3(kOsThreads), 0, s, io, n,
                         n_dev, p, words, gather_src, gather_tiles, gather_dst, gather_dst2, err);
    else
      hipLaunchKernelGGL(radix_onesweep<kOsRowsBig>, dim3(grid), dim3(kOsThreads), 0, s, io, n,
                         n_dev, p, words, gather_src, gather_tiles, gather_dst, gather_dst2, err);
  }
  return (passes - 1) & 1;
}

void launch_zero_list(const FillList &f, hipStream_t s) {
  int64_t total = 0;
  for (int a = 0; a < FillList::kMax; ++a) total += f.n[a] > 0 ? f.n[a] : 0;
  if (total == 0) return;
  FillList g = f;
  for (int a = 0; a < FillList::kMax; ++a)
    if (g.n[a] < 0) g.n[a] = 0;
  const int64_t blocks = std::min<int64_t>((total + 255) / 256, 1024);
  hipLaunchKernelGGL(zero_list_kernel, dim3((unsigned)blocks), dim3(256), 0, s, g, total);
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
  // a capacity-sized count (D_dev given) strides over a bounded grid
  const int64_t blocks = D_dev ? std::min<int64_t>((D + 255) / 256, 8192) : (D + 255) / 256;
  hipLaunchKernelGGL(ranges_kernel, dim3((unsigned)blocks), dim3(256), 0, s, keys, D, D_dev,
                     ranges);
}

}  // namespace hgs
