// Device memory held in the library's code object instead of hipMalloc'd
// buffers:
//   * a pool for the kernels' constant tables (colex rank / unrank tables,
//     EdgeJoin slot maps, NodeJoin split maps), filled once per device and k;
//   * `scratch`, the work memory of cc_count_static, the counting call that
//     allocates nothing: every device buffer of its solve is carved from it.
// Both live as long as the process on every device the library runs on.  In
// host code the arrays' names are host-side stand-ins, never device
// addresses: their device addresses come from hipGetSymbolAddress, once per
// device with that device current, and only those addresses are used.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>

#include "cc_internal.h"

namespace cc {

namespace {

constexpr size_t kTablePoolBytes = (size_t)2 << 20;  // every table of k = 3..12: about 0.65 MB
static __device__ __align__(256) uint8_t table_pool[kTablePoolBytes];
static __device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

struct PerDevice {
  uint8_t *tables = nullptr;  // device address of table_pool
  size_t tables_used = 0;
  uint8_t *scratch = nullptr;  // device address of scratch
};
std::mutex g_mu;
std::map<int, PerDevice> g_dev;
std::map<int, std::unique_ptr<std::mutex>> g_scratch_mu;

}  // namespace

void *table_pool_alloc(size_t bytes) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  PerDevice &P = g_dev[dev];
  if (!P.tables) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(table_pool)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return nullptr;
    }
    P.tables = (uint8_t *)p;
  }
  const size_t b = (bytes + 255) & ~(size_t)255;
  if (P.tables_used + b > kTablePoolBytes) return nullptr;
  void *out = P.tables + P.tables_used;
  P.tables_used += b;
  return out;
}

uint8_t *static_scratch(int dev) {
  std::lock_guard<std::mutex> lk(g_mu);
  PerDevice &P = g_dev[dev];
  if (!P.scratch) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      fail(CC_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    P.scratch = (uint8_t *)p;
  }
  return P.scratch;
}

std::mutex &static_scratch_lock(int dev) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto &m = g_scratch_mu[dev];
  if (!m) m.reset(new std::mutex);
  return *m;
}

}  // namespace cc
