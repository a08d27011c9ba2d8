// Statistics of a caller's field with no handle and no allocation (at_field_stats_noalloc).
//
// The kernels are those of at_stats: per-block FP64 partials with synchronous central derivatives,
// then the fixed-order two-level reduction.  Their scratch - the block partials, the level-1 rows
// and the reduced sums - lives in the file-scope device array below instead of a workspace, so the
// call allocates nothing.  Each device that runs the library holds its own copy of the array
// (at its own address, looked up once per device with hipGetSymbolAddress) until the process
// ends; every call on a device shares it and leaves the last call's contents there.  Each call
// overwrites every element it reads before reading it (every statistics block writes its partial,
// every level-1 workgroup its row), so nothing needs clearing between calls.
#include <mutex>

#include "sim_internal.h"

using namespace atns;

// Largest number of statistics blocks (64 x 4 points of one z plane each): 256^3 needs 65536.
constexpr int64_t kNoallocMaxBlocks = 65536;
constexpr size_t kScratchDoubles = (size_t)kNoallocMaxBlocks * kNStat + kStatOutBytes / sizeof(double);
static_assert(AT_STATS_NOALLOC_MAX_BLOCKS == kNoallocMaxBlocks, "header and library limits agree");

// In host code `scratch` names a host-side stand-in, not device memory: host code uses only the
// per-device address that hipGetSymbolAddress returns for it.
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// The device address of this device's copy of `scratch` (looked up on its first use here).
int scratch_of_device(double** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(AT_E_INVAL, "device index beyond the library's table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(AT_E_HIP, "hipGetSymbolAddress returned a null address for the statistics scratch");
    g_scratch_ptr[dev] = (double*)p;
  }
  *out = g_scratch_ptr[dev];
  return AT_OK;
}

template <typename T>
int field_stats(const at_config* cfg, const void* dev_q, at_stats_t* dev_out, hipStream_t stream, double* sc) {
  const Geom g = make_geom(cfg);
  double* part = sc;
  double* out = sc + (size_t)kNoallocMaxBlocks * kNStat;
  HIP_TRY(launch_stats<T>(g, coef_of<T>(*cfg), (const T*)dev_q, part, out, nullptr, 0, cfg->gamma, stream, nullptr));
  const double vol = (kTwoPi / cfg->n[0]) * (kTwoPi / cfg->n[1]) * (kTwoPi / cfg->n[2]);
  HIP_TRY(launch_stats_record(out, dev_out, (double)g.npts, vol, cfg->gamma, cfg->gas_r, stream));
  return AT_OK;
}

}  // namespace

extern "C" {

int at_field_stats_noalloc(const at_config* cfg, const void* dev_q, at_stats_t* dev_out, void* hip_stream) {
  int rc = validate(cfg);
  if (rc) return rc;
  if (!dev_q || !dev_out) return fail(AT_E_INVAL, "NULL field or output pointer");
  const Geom g = make_geom(cfg);
  if (stats_blocks(g) > kNoallocMaxBlocks)
    return fail(AT_E_INVAL, "grid needs more statistics blocks (ceil(nx/64) ceil(ny/4) nz) than the "
                            "allocation-free scratch holds (65536)");
  double* sc = nullptr;
  rc = scratch_of_device(&sc);
  if (rc) return rc;
  const hipStream_t st = (hipStream_t)hip_stream;
  return cfg->precision == AT_FP32 ? field_stats<float>(cfg, dev_q, dev_out, st, sc)
                                   : field_stats<double>(cfg, dev_q, dev_out, st, sc);
}

}  // extern "C"
