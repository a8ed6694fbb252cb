// Allocation-free variant of the matrix-element stage: the grouped pair
// contraction writes H and S into caller-owned device buffers, and the one
// piece of device memory beyond inputs and outputs that its kernels read --
// the pair task list -- is staged in a file-scope device array instead of a
// hipMalloc'd buffer.
//
// The array is a host-side stand-in in host code: its device address is
// resolved once per device with hipGetSymbolAddress (noalloc_init, called by
// ofm_create with the device current) and only that address is ever handed
// to kernels or copies.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "ofm_internal.h"

namespace {

// one per GPU the library runs on, held until the process ends
static __device__ __align__(256) unsigned char scratch[OFM_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

}  // namespace

namespace ofm {

void noalloc_init(int device) {
  OFM_REQUIRE(device >= 0 && device < kMaxDevices, OFM_E_INVALID,
              "device index above the library's limit of 64");
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_scratch[device]) return;
  void* p = nullptr;
  OFM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  OFM_REQUIRE(p != nullptr, OFM_E_DEVICE,
              "hipGetSymbolAddress returned no address for the scratch array");
  g_scratch[device] = p;
}

}  // namespace ofm

using namespace ofm;

extern "C" ofm_status ofm_matrix_elements_noalloc(ofm_ctx* c, ofm_frags* f,
                                                  double* H_dev,
                                                  double* S_dev) {
  if (!c) return OFM_E_INVALID;
  c->err.clear();
  const bool prof = c->profiling;
  try {
    OFM_REQUIRE(f && f->ctx == c && H_dev && S_dev, OFM_E_INVALID,
                "bad arguments");
    OFM_REQUIRE(f->have_states, OFM_E_STATE,
                "matrix elements need fragment states (solve or set_states)");
    const size_t need = sizeof(PairTask) * f->pair_tasks.size();
    OFM_REQUIRE(need <= (size_t)OFM_NOALLOC_SCRATCH_BYTES, OFM_E_INVALID,
                "the pair task list (" + std::to_string(f->pair_tasks.size()) +
                    " tasks, " + std::to_string(need) +
                    " bytes) exceeds the allocation-free scratch of " +
                    std::to_string((long long)OFM_NOALLOC_SCRATCH_BYTES) +
                    " bytes");
    OFM_HIP(hipSetDevice(c->device));
    for (double* p : {H_dev, S_dev}) {
      hipPointerAttribute_t a;
      const hipError_t e = hipPointerGetAttributes(&a, p);
      if (e != hipSuccess) (void)hipGetLastError();
      OFM_REQUIRE(e == hipSuccess && a.type == hipMemoryTypeDevice,
                  OFM_E_INVALID, "H_dev and S_dev must be device memory");
    }
    void* p = nullptr;
    {
      std::lock_guard<std::mutex> lk(g_mu);
      p = c->device < kMaxDevices ? g_scratch[c->device] : nullptr;
    }
    OFM_REQUIRE(p != nullptr, OFM_E_STATE,
                "the scratch array of this device was not resolved");
    // no timing brackets: their events are not needed here
    c->profiling = false;
    // no timing runs here: the variant is the pinned, cached or default one
    run_pair_elements(c, f, static_cast<PairTask*>(p), H_dev, S_dev, false);
    c->profiling = prof;
    return OFM_OK;
  } catch (const Error& e) {
    c->profiling = prof;
    c->err = e.msg;
    return e.code;
  } catch (const std::exception& e) {
    c->profiling = prof;
    c->err = e.what();
    return OFM_E_INVALID;
  }
}
