// Allocation-free execution support: a file-scope device array that holds the
// descriptor tables of tcfft_exec_many_static, and a kernel that writes those
// tables from its by-value arguments (no host staging memory, no device
// allocation).
//
// In host code the array's name is only a host-side stand-in: the device
// address of each GPU's copy comes from hipGetSymbolAddress, taken once per
// device (with that device current) and kept in g_ptr; only that address is
// ever passed to kernels.
#include <algorithm>
#include <mutex>

#include "../../include/tcfft.h"
#include "kernels.h"

namespace tcfft {

constexpr size_t kStaticScratchBytes = TCFFT_STATIC_SCRATCH_BYTES;

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices];
}  // namespace

hipError_t static_scratch(void** out, size_t* bytes) {
  *out = nullptr;
  *bytes = 0;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  *bytes = kStaticScratchBytes;
  return hipSuccess;
}

// Up to kWords 32-bit words carried in the kernel arguments.
constexpr int kWords = 240;
struct WordChunk {
  uint32_t* dst;
  uint32_t n;
  uint32_t words[kWords];
};

__global__ __launch_bounds__(256) void write_words_kernel(WordChunk c) {
  for (uint32_t i = threadIdx.x; i < c.n; i += 256) c.dst[i] = c.words[i];
}

hipError_t launch_write_words(void* dst, const void* src, size_t bytes, hipStream_t s) {
  if (bytes % 4 != 0) return hipErrorInvalidValue;
  const uint32_t* w = (const uint32_t*)src;
  const size_t total = bytes / 4;
  for (size_t off = 0; off < total; off += kWords) {
    WordChunk c;
    c.dst = (uint32_t*)dst + off;
    c.n = (uint32_t)std::min<size_t>(kWords, total - off);
    for (uint32_t i = 0; i < c.n; ++i) c.words[i] = w[off + i];
    hipLaunchKernelGGL(write_words_kernel, dim3(1), dim3(256), 0, s, c);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace tcfft
