// Device-wide exclusive prefix sums (reduce-then-scan, three launches).
// Used for radix-sort digit offsets and for the per-tile work plan.
#include "sfk_device.h"

namespace sfk {

static constexpr int kScanNT = 256;
static constexpr int kScanItems = 16;
static constexpr int kScanTile = kScanNT * kScanItems;

template <typename TI, typename TO>
__global__ __launch_bounds__(kScanNT) void k_scan_reduce(const TI* __restrict__ in, int64_t n,
                                                         TO* __restrict__ bsum) {
  __shared__ TO lds[kScanNT / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  TO s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t g = base + (int64_t)i * kScanNT + threadIdx.x;
    if (g < n) s += (TO)in[g];
  }
  s = wave_sum(s);
  if (lane_id() == 0) lds[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    TO t = 0;
    for (int w = 0; w < kScanNT / 64; ++w) t += lds[w];
    bsum[blockIdx.x] = t;
  }
}

// One block: exclusive scan of the block sums in place; writes the total.
template <typename TO>
__global__ __launch_bounds__(kScanNT) void k_scan_blocks(TO* __restrict__ bsum, int64_t nb,
                                                         TO* __restrict__ total) {
  __shared__ TO lds[kScanNT / 64];
  TO carry = 0;
  for (int64_t base = 0; base < nb; base += kScanNT) {
    const int64_t g = base + threadIdx.x;
    TO v = g < nb ? bsum[g] : (TO)0;
    TO tot;
    TO ex = block_excl_scan<kScanNT>(v, &tot, lds);
    if (g < nb) bsum[g] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0 && total) *total = carry;
}

// Each thread scans kScanItems consecutive elements of the block's tile.
template <typename TI, typename TO>
__global__ __launch_bounds__(kScanNT) void k_scan_apply(const TI* __restrict__ in,
                                                        TO* __restrict__ out, int64_t n,
                                                        const TO* __restrict__ bsum) {
  __shared__ TO lds[kScanNT / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  TO v[kScanItems];
  TO s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t g = base + i;
    v[i] = g < n ? (TO)in[g] : (TO)0;
    s += v[i];
  }
  TO tot;
  TO ex = block_excl_scan<kScanNT>(s, &tot, lds) + bsum[blockIdx.x];
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t g = base + i;
    if (g < n) out[g] = ex;
    ex += v[i];
  }
}

template <typename TO>
__global__ void k_store_zero(TO* p) { *p = 0; }

size_t scan_tmp_bytes(int64_t n) {
  const int64_t nb = (n + kScanTile - 1) / kScanTile;
  return (size_t)(nb + 1) * sizeof(int64_t) + 256;
}

template <typename TI, typename TO>
static hipError_t scan_impl(const TI* in, TO* out, int64_t n, TO* total, void* tmp,
                            size_t tmp_bytes, hipStream_t s) {
  const int64_t nb = (n + kScanTile - 1) / kScanTile;
  if (n <= 0) {
    if (total) hipLaunchKernelGGL((k_store_zero<TO>), dim3(1), dim3(1), 0, s, total);
    return hipGetLastError();
  }
  if ((size_t)(nb + 1) * sizeof(TO) > tmp_bytes) return hipErrorInvalidValue;
  TO* bsum = (TO*)tmp;
  hipLaunchKernelGGL((k_scan_reduce<TI, TO>), dim3((unsigned)nb), dim3(kScanNT), 0, s, in, n, bsum);
  hipLaunchKernelGGL((k_scan_blocks<TO>), dim3(1), dim3(kScanNT), 0, s, bsum, nb, total);
  hipLaunchKernelGGL((k_scan_apply<TI, TO>), dim3((unsigned)nb), dim3(kScanNT), 0, s, in, out, n,
                     (const TO*)bsum);
  return hipGetLastError();
}

hipError_t scan_exclusive_i32_i64(const int32_t* in, int64_t* out, int64_t n, int64_t* total,
                                  void* tmp, size_t tmp_bytes, hipStream_t s) {
  return scan_impl<int32_t, int64_t>(in, out, n, total, tmp, tmp_bytes, s);
}

hipError_t scan_exclusive_u32(const uint32_t* in, uint32_t* out, int64_t n, void* tmp,
                              size_t tmp_bytes, hipStream_t s) {
  return scan_impl<uint32_t, uint32_t>(in, out, n, (uint32_t*)nullptr, tmp, tmp_bytes, s);
}

}  // namespace sfk
