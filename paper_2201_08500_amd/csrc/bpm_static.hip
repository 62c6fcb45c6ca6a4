// bpm_propagate_noalloc: bpm_propagate for callers that cannot allocate
// device memory.  The deformation table exp(i h u) -- and the plan's
// per-slice constants and crystal mask while the plan has not uploaded them
// itself -- live in one file-scope device array of fixed size instead of
// stream-ordered allocations.  The kernels are the ones bpm_propagate runs,
// so the results are bitwise the same.

#include <cstring>
#include <mutex>
#include <string>

#include "bpm_internal.h"

namespace {

constexpr size_t kStaticBytes = size_t(BPM_NOALLOC_MAX_BYTES);

// One copy per device, held until the process ends.  Host code must never
// pass this name to a kernel or a copy: on the host it is only a stand-in
// for the symbol, and its device address comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[kStaticBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned char* g_addr[kMaxDevices] = {};   // device address of scratch per device

// Address of the current device's copy of scratch, looked up once per device
// (with that device current).
int scratch_address(unsigned char** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess)
    return bpm::set_error(BPM_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices)
    return bpm::set_error(BPM_EUNSUPPORTED, "device index beyond the static workspace table");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_addr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return bpm::set_error(BPM_EHIP, std::string("hipGetSymbolAddress(static workspace): ") +
                                          hipGetErrorString(e));
    g_addr[dev] = static_cast<unsigned char*>(ptr);
  }
  *out = g_addr[dev];
  return BPM_OK;
}

size_t round256(size_t n) { return (n + 255) & ~size_t(255); }

}  // namespace

extern "C" int bpm_propagate_noalloc(const bpm_plan* cp, const void* E0_in,
                                     const double* u_field, void* E0_out, void* Eh_out,
                                     void* stream) {
  bpm::clear_error();
  if (!cp) return bpm::set_error(BPM_EINVAL, "plan is NULL");
  if (!E0_in || !E0_out || !Eh_out)
    return bpm::set_error(BPM_EINVAL, "E0_in, E0_out and Eh_out must be non-NULL");
  if (E0_in == E0_out || E0_in == Eh_out || E0_out == Eh_out)
    return bpm::set_error(BPM_EINVAL, "output buffers must not alias each other or E0_in");
  if (cp->three_d)
    return bpm::set_error(BPM_EUNSUPPORTED, "bpm_propagate_noalloc is not available for 3D plans");
  bpm_plan* p = const_cast<bpm_plan*>(cp);
  int rc = bpm::plan_freeze_host(p);
  if (rc) return rc;
  const bpm::SliceConst* dev_sc = nullptr;
  const unsigned char* dev_mask = nullptr;
  {
    std::lock_guard<std::mutex> lock(p->mu);
    dev_sc = p->dev_sc;
    dev_mask = p->dev_mask;
  }
  const bool masked = !p->mask.empty();
  // Layout: [slice constants][crystal mask][deformation table], each part
  // only when needed, each 256-byte aligned.
  const size_t sc_bytes = dev_sc ? 0 : round256(sizeof(bpm::SliceConst) * size_t(p->Nomega));
  const size_t mask_bytes = (masked && !dev_mask) ? round256(p->mask.size()) : 0;
  const size_t cell = p->precision == BPM_PREC_FP64 ? 16 : 8;
  const size_t table_bytes = u_field ? size_t(p->Nx) * size_t(p->Nz) * cell : 0;
  const size_t need = sc_bytes + mask_bytes + table_bytes;
  if (need > kStaticBytes)
    return bpm::set_error(
        BPM_EINVAL, "problem needs " + std::to_string(need) + " B of workspace, more than the " +
                        std::to_string(kStaticBytes) +
                        " B static workspace of bpm_propagate_noalloc (use bpm_propagate_ws)");
  unsigned char* base = nullptr;
  rc = scratch_address(&base);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  unsigned char* sc_at = base;
  unsigned char* mask_at = base + sc_bytes;
  unsigned char* table_at = base + sc_bytes + mask_bytes;
  if (!dev_sc) {
    hipError_t e = hipMemcpyAsync(sc_at, p->sc.data(), sizeof(bpm::SliceConst) * p->sc.size(),
                                  hipMemcpyHostToDevice, s);
    if (e != hipSuccess)
      return bpm::set_error(BPM_EHIP, std::string("plan constants to the static workspace: ") +
                                          hipGetErrorString(e));
    dev_sc = reinterpret_cast<const bpm::SliceConst*>(sc_at);
  }
  if (masked && !dev_mask) {
    hipError_t e = hipMemcpyAsync(mask_at, p->mask.data(), p->mask.size(),
                                  hipMemcpyHostToDevice, s);
    if (e != hipSuccess)
      return bpm::set_error(BPM_EHIP, std::string("crystal mask to the static workspace: ") +
                                          hipGetErrorString(e));
    dev_mask = mask_at;
  }
  if (u_field) {
    rc = bpm::launch_deform(p->precision, p->Nx, p->Nz, p->h, u_field, table_at, s);
    if (rc) return bpm::set_error(rc, "deformation pre-pass launch failed");
  }
  bpm::MarchParams m =
      bpm::plan_march_params(p, E0_in, u_field ? table_at : nullptr, E0_out, Eh_out);
  m.sc = dev_sc;
  m.mask = masked ? dev_mask : nullptr;
  rc = bpm::launch_march(p->precision, p->Nx, bpm::plan_schedule_of(p), p->split_order,
                         p->Nomega, m, s);
  if (rc == BPM_EUNSUPPORTED) return bpm::set_error(rc, "unsupported size/precision");
  if (rc) return bpm::set_error(rc, "march kernel launch failed");
  return BPM_OK;
}
