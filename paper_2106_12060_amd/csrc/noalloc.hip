// CountSketch without any device allocation, for callers that cannot
// allocate (code under HIP graph capture, tight serving loops, harnesses
// that forbid hipMalloc).  Same result as srp_countsketch; its scratch
// (bucket counts, offsets, cursors and the two row lists of the bucket
// sort) lives in one file-scope device array per GPU instead of the
// stream-ordered pool.
#include "common.hpp"
#include "kernels.hpp"

#include <mutex>

namespace srp {

// Largest sizes the array serves: rows and buckets.
constexpr int64_t kNoAllocMaxRows = int64_t(1) << 22;
constexpr int kNoAllocMaxBuckets = 1 << 20;
// Exactly what countsketch_run takes from its arena at the largest sizes
// (three (s + 1)-int tables and two n-int lists, each rounded to 256 B).
constexpr size_t kNoAllocScratchBytes =
    3 * ((sizeof(int) * (size_t(kNoAllocMaxBuckets) + 1) + 255) & ~size_t(255)) +
    2 * ((sizeof(int) * size_t(kNoAllocMaxRows) + 255) & ~size_t(255));

// 44 MiB per GPU, held from the first launch on that GPU until the process
// ends.  Host code never uses this name as an address: the device address
// comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

static int scratch_address(void** out) {
  static std::mutex mu;
  static void* addr[64] = {};
  int dev = 0;
  SRP_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) {
    set_error("countsketch_noalloc: device %d out of range", dev);
    return SRP_EINVAL;
  }
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    SRP_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) {
      set_error("countsketch_noalloc: no device address for the scratch array");
      return SRP_EDEVICE;
    }
    addr[dev] = p;
  }
  *out = addr[dev];
  return SRP_OK;
}

}  // namespace srp

using namespace srp;

extern "C" int srp_countsketch_noalloc(const void* A, int dtype, int64_t n, int d, int s, uint64_t seed, void* out,
                                       void* stream) {
  clear_error();
  SRP_REQUIRE(A && out, "null pointer argument");
  SRP_REQUIRE(n >= 1 && d >= 1 && s >= 1, "bad sizes");
  SRP_REQUIRE(n <= kNoAllocMaxRows, "countsketch_noalloc: n = %lld rows exceeds the scratch limit of %lld",
              (long long)n, (long long)kNoAllocMaxRows);
  SRP_REQUIRE(s <= kNoAllocMaxBuckets, "countsketch_noalloc: s = %d buckets exceeds the scratch limit of %d", s,
              kNoAllocMaxBuckets);
  SRP_REQUIRE(dtype == SRP_F64 || dtype == SRP_F32 || dtype == SRP_BF16 || dtype == SRP_FP8E4M3, "bad dtype %d",
              dtype);
  void* base = nullptr;
  SRP_TRY(scratch_address(&base));
  Arena ar{(char*)base, kNoAllocScratchBytes, 0};
  return countsketch_run(A, dtype, n, d, s, seed, out, ar, (hipStream_t)stream);
}
