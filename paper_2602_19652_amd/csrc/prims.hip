// Device primitives: exclusive scan (u64) and stable LSD radix sort (4-bit digits).
// Both take the element count either from the host or from device memory, so that they
// can run behind kernels whose output size is only known on the device (no host sync).
#include "internal.hpp"

namespace et {

namespace {

constexpr int SB = 256;          // threads per block
constexpr int SI = 8;            // items per thread
constexpr int TILE = SB * SI;    // elements per block

__device__ inline int64_t get_n(int64_t n_host, const int64_t* n_dev) { return n_dev ? *n_dev : n_host; }

// Inclusive scan of one value per lane across the 64-lane wave.
template <typename T>
__device__ inline T wave_incl_scan(T v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    T o = __shfl_up(v, d, 64);
    if (lane >= d) v += o;
  }
  return v;
}

// Exclusive scan across the block (SB threads); returns the block total in *total.
template <typename T>
__device__ inline T block_excl_scan(T v, T* total) {
  __shared__ T wsum[SB / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  T inc = wave_incl_scan(v);
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  T off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < SB / 64; ++i) {
    if (i < w) off += wsum[i];
    tot += wsum[i];
  }
  __syncthreads();
  *total = tot;
  return off + inc - v;
}

__global__ void k_scan_reduce(const uint64_t* __restrict__ in, int64_t n_host, const int64_t* n_dev,
                              uint64_t* __restrict__ bsum) {
  const int64_t n = get_n(n_host, n_dev);
  const int64_t base = (int64_t)blockIdx.x * TILE;
  if (base >= n) return;
  uint64_t s = 0;
#pragma unroll
  for (int i = 0; i < SI; ++i) {
    int64_t idx = base + (int64_t)i * SB + threadIdx.x;
    if (idx < n) s += in[idx];
  }
  uint64_t tot;
  block_excl_scan<uint64_t>(s, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// Single block: exclusive scan of the block sums, in chunks with a running carry.
__global__ void k_scan_blocks(uint64_t* __restrict__ bsum, int64_t n_host, const int64_t* n_dev,
                              uint64_t* __restrict__ total) {
  const int64_t n = get_n(n_host, n_dev);
  const int64_t nb = (n + TILE - 1) / TILE;
  uint64_t carry = 0;
  for (int64_t c = 0; c < nb; c += SB) {
    int64_t i = c + threadIdx.x;
    uint64_t v = i < nb ? bsum[i] : 0;
    uint64_t tot;
    uint64_t ex = block_excl_scan<uint64_t>(v, &tot);
    if (i < nb) bsum[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0 && total) *total = carry;
}

__global__ void k_scan_apply(const uint64_t* __restrict__ in, uint64_t* __restrict__ out, int64_t n_host,
                             const int64_t* n_dev, const uint64_t* __restrict__ bsum) {
  const int64_t n = get_n(n_host, n_dev);
  const int64_t base = (int64_t)blockIdx.x * TILE;
  if (base >= n) return;
  // thread t owns the contiguous items [base + t*SI, base + t*SI + SI)
  uint64_t v[SI];
  uint64_t s = 0;
#pragma unroll
  for (int i = 0; i < SI; ++i) {
    int64_t idx = base + (int64_t)threadIdx.x * SI + i;
    v[i] = idx < n ? in[idx] : 0;
    s += v[i];
  }
  uint64_t tot;
  uint64_t ex = block_excl_scan<uint64_t>(s, &tot) + bsum[blockIdx.x];
#pragma unroll
  for (int i = 0; i < SI; ++i) {
    int64_t idx = base + (int64_t)threadIdx.x * SI + i;
    if (idx < n) out[idx] = ex;
    ex += v[i];
  }
}

// Short arrays (at most SCAN_ONE_MAX elements, e.g. a radix pass's digit counts): one
// workgroup scans the tiles in turn with a running carry, one launch instead of three.  Past
// two tiles the three-launch scan, whose workgroups run in parallel, is faster (measured at
// 16384 elements).  The count is clamped to the caller's bound n_max.
constexpr int64_t SCAN_ONE_MAX = 2 * TILE;

__global__ void k_scan_one(const uint64_t* __restrict__ in, uint64_t* __restrict__ out, int64_t n_host,
                           const int64_t* n_dev, int64_t n_max, uint64_t* __restrict__ total) {
  int64_t n = get_n(n_host, n_dev);
  n = n < n_max ? n : n_max;
  uint64_t carry = 0;
  for (int64_t base = 0; base < n; base += TILE) {
    // thread t owns the contiguous items [base + t*SI, base + t*SI + SI)
    uint64_t v[SI];
    uint64_t s = 0;
#pragma unroll
    for (int i = 0; i < SI; ++i) {
      const int64_t idx = base + (int64_t)threadIdx.x * SI + i;
      v[i] = idx < n ? in[idx] : 0;
      s += v[i];
    }
    uint64_t tot;
    uint64_t ex = block_excl_scan<uint64_t>(s, &tot) + carry;
#pragma unroll
    for (int i = 0; i < SI; ++i) {
      const int64_t idx = base + (int64_t)threadIdx.x * SI + i;
      if (idx < n) out[idx] = ex;
      ex += v[i];
    }
    carry += tot;
  }
  if (threadIdx.x == 0 && total) *total = carry;
}

// ------------------------------------------------------------------ radix sort

constexpr int RBITS = 4;
constexpr int RADIX = 1 << RBITS;

template <typename K>
__global__ void k_radix_hist(const K* __restrict__ keys, int64_t n_host, const int64_t* n_dev, int shift,
                             uint64_t* __restrict__ hist, int64_t nblocks_max) {
  const int64_t n = get_n(n_host, n_dev);
  __shared__ uint32_t cnt[RADIX];
  if (threadIdx.x < RADIX) cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * TILE;
#pragma unroll
  for (int i = 0; i < SI; ++i) {
    int64_t idx = base + (int64_t)i * SB + threadIdx.x;
    if (idx < n) atomicAdd(&cnt[(uint32_t)(keys[idx] >> shift) & (RADIX - 1)], 1u);
  }
  __syncthreads();
  // digit-major layout so that one exclusive scan yields the scatter bases
  if (threadIdx.x < RADIX) hist[(int64_t)threadIdx.x * nblocks_max + blockIdx.x] = cnt[threadIdx.x];
}

template <typename K>
__global__ void k_radix_scatter(const K* __restrict__ kin, const int32_t* __restrict__ vin, K* __restrict__ kout,
                                int32_t* __restrict__ vout, int64_t n_host, const int64_t* n_dev, int shift,
                                const uint64_t* __restrict__ offs, int64_t nblocks_max) {
  const int64_t n = get_n(n_host, n_dev);
  const int64_t base = (int64_t)blockIdx.x * TILE;
  if (base >= n) return;
  __shared__ uint32_t pre[RADIX * SB];   // [digit][thread] counts, then exclusive offsets
  K k[SI];
  int32_t v[SI];
  uint32_t dg[SI];
  uint32_t c[RADIX];
#pragma unroll
  for (int d = 0; d < RADIX; ++d) c[d] = 0;
#pragma unroll
  for (int i = 0; i < SI; ++i) {
    int64_t idx = base + (int64_t)threadIdx.x * SI + i;   // contiguous items keep the sort stable
    if (idx < n) {
      k[i] = kin[idx];
      v[i] = vin[idx];
      dg[i] = (uint32_t)(k[i] >> shift) & (RADIX - 1);
    } else {
      dg[i] = RADIX;  // padding
    }
#pragma unroll
    for (int d = 0; d < RADIX; ++d) c[d] += (dg[i] == (uint32_t)d);
  }
#pragma unroll
  for (int d = 0; d < RADIX; ++d) pre[d * SB + threadIdx.x] = c[d];
  __syncthreads();
  // per digit: exclusive scan over threads (each thread scans one digit row segment)
  // RADIX rows of SB entries: thread t handles row (t / (SB/RADIX)), segment of RADIX entries
  {
    const int row = threadIdx.x / (SB / RADIX);
    const int seg = threadIdx.x % (SB / RADIX);
    uint32_t* r = pre + row * SB + seg * RADIX;
    uint32_t s = 0;
    uint32_t tmp[RADIX];
#pragma unroll
    for (int i = 0; i < RADIX; ++i) { tmp[i] = s; s += r[i]; }
    // scan of segment sums within the row: SB/RADIX = 16 segments, lanes of the same row are contiguous
    uint32_t segsum = s;
    uint32_t inc = segsum;
#pragma unroll
    for (int d = 1; d < SB / RADIX; d <<= 1) {
      uint32_t o = __shfl_up(inc, d, SB / RADIX);
      if (seg >= d) inc += o;
    }
    uint32_t ex = inc - segsum;
#pragma unroll
    for (int i = 0; i < RADIX; ++i) r[i] = tmp[i] + ex;
  }
  __syncthreads();
  uint32_t run[RADIX];
#pragma unroll
  for (int d = 0; d < RADIX; ++d) run[d] = 0;
#pragma unroll
  for (int i = 0; i < SI; ++i) {
    if (dg[i] < RADIX) {
      const uint32_t d = dg[i];
      uint64_t pos = offs[(int64_t)d * nblocks_max + blockIdx.x] + pre[d * SB + threadIdx.x];
      uint32_t add = 0;
#pragma unroll
      for (int e = 0; e < RADIX; ++e) add += (e == (int)d) ? run[e] : 0u;
      pos += add;
      kout[pos] = k[i];
      vout[pos] = v[i];
#pragma unroll
      for (int e = 0; e < RADIX; ++e) run[e] += (e == (int)d);
    }
  }
}

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace

size_t scan_temp_bytes(int64_t n_max) { return (size_t)(ceil_div(n_max > 0 ? n_max : 1, TILE) + 1) * sizeof(uint64_t); }

void scan_exclusive_u64(const uint64_t* in, uint64_t* out, int64_t n_host, const int64_t* n_dev, int64_t n_max,
                        uint64_t* total, void* temp, hipStream_t s) {
  if (n_max <= 0) n_max = 1;
  if (n_max <= SCAN_ONE_MAX) {
    k_scan_one<<<1, SB, 0, s>>>(in, out, n_host, n_dev, n_max, total);
    ET_HIP(hipGetLastError());
    return;
  }
  const int64_t nb = ceil_div(n_max, TILE);
  uint64_t* bsum = (uint64_t*)temp;
  k_scan_reduce<<<(unsigned)nb, SB, 0, s>>>(in, n_host, n_dev, bsum);
  k_scan_blocks<<<1, SB, 0, s>>>(bsum, n_host, n_dev, total);
  k_scan_apply<<<(unsigned)nb, SB, 0, s>>>(in, out, n_host, n_dev, bsum);
  ET_HIP(hipGetLastError());
}

size_t sort_temp_bytes(int64_t n, int key_bytes) {
  if (n <= 0) n = 1;
  const int64_t nb = ceil_div(n, TILE);
  size_t b = 0;
  b += (size_t)n * key_bytes + 256;          // key ping-pong
  b += (size_t)n * sizeof(int32_t) + 256;    // value ping-pong
  b += (size_t)RADIX * nb * sizeof(uint64_t) * 2 + 256;   // histogram + offsets
  b += scan_temp_bytes(RADIX * nb) + 256;
  return b;
}

template <typename K>
static void radix_sort_impl(K* keys, int32_t* vals, int64_t n_host, const int64_t* n_dev, int64_t n_max, int bits,
                            void* temp, hipStream_t s) {
  if (n_max <= 0) return;
  const int64_t nb = ceil_div(n_max, TILE);
  char* t = (char*)temp;
  auto take = [&](size_t bytes) { char* p = t; t += (bytes + 255) / 256 * 256; return (void*)p; };
  K* k2 = (K*)take((size_t)n_max * sizeof(K));
  int32_t* v2 = (int32_t*)take((size_t)n_max * sizeof(int32_t));
  uint64_t* hist = (uint64_t*)take((size_t)RADIX * nb * sizeof(uint64_t));
  uint64_t* offs = (uint64_t*)take((size_t)RADIX * nb * sizeof(uint64_t));
  void* stemp = take(scan_temp_bytes(RADIX * nb));
  K* ka = keys; int32_t* va = vals; K* kb = k2; int32_t* vb = v2;
  const int passes = (bits + RBITS - 1) / RBITS;
  for (int p = 0; p < passes; ++p) {
    const int shift = p * RBITS;
    k_radix_hist<K><<<(unsigned)nb, SB, 0, s>>>(ka, n_host, n_dev, shift, hist, nb);
    scan_exclusive_u64(hist, offs, RADIX * nb, nullptr, RADIX * nb, nullptr, stemp, s);
    k_radix_scatter<K><<<(unsigned)nb, SB, 0, s>>>(ka, va, kb, vb, n_host, n_dev, shift, offs, nb);
    ET_HIP(hipGetLastError());
    K* tk = ka; ka = kb; kb = tk;
    int32_t* tv = va; va = vb; vb = tv;
  }
  if (ka != keys) {
    // odd number of passes: copy back (n may live on the device: copy n_max)
    ET_HIP(hipMemcpyAsync(keys, ka, (size_t)n_max * sizeof(K), hipMemcpyDeviceToDevice, s));
    ET_HIP(hipMemcpyAsync(vals, va, (size_t)n_max * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  }
}

void radix_sort_u32(uint32_t* keys, int32_t* vals, int64_t n, int bits, void* temp, hipStream_t s) {
  radix_sort_impl<uint32_t>(keys, vals, n, nullptr, n, bits, temp, s);
}

void radix_sort_u64(uint64_t* keys, int32_t* vals, int64_t n_host, const int64_t* n_dev, int64_t n_max, int bits,
                    void* temp, hipStream_t s) {
  radix_sort_impl<uint64_t>(keys, vals, n_host, n_dev, n_max, bits, temp, s);
}

}  // namespace et
