// Host-memory stand-ins for the few HIP runtime calls and library internals that the plan
// builder (plan.cpp) uses, so that its host code (stencil weights, generating-array
// spectra, D^e tables, frame spectra, preconditioner symbols, constraint and broken-bond
// validation, crack -> bonds, surface factors) runs in a CPU process under AddressSanitizer
// and UndefinedBehaviorSanitizer.  "Device" buffers are host allocations here.  Test
// infrastructure: linked only into tests/sanitize/plan_host_driver.cpp.
#include <cstdlib>
#include <cstring>

#include "../../paper_2301_11828_amd/csrc/common.hpp"

extern "C" {
hipError_t hipMalloc(void **ptr, size_t size) {
    *ptr = std::calloc(1, size ? size : 1);
    return *ptr ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void *ptr) {
    std::free(ptr);
    return hipSuccess;
}
hipError_t hipMemcpy(void *dst, const void *src, size_t n, hipMemcpyKind) {
    std::memcpy(dst, src, n);
    return hipSuccess;
}
hipError_t hipGetDevice(int *dev) {
    *dev = 0;
    return hipSuccess;
}
hipError_t hipDeviceSynchronize(void) { return hipSuccess; }
const char *hipGetErrorString(hipError_t) { return "host stand-in"; }
}

namespace msb {
// the launch configuration is the kernels' business: a fixed valid-looking default, and
// every configuration accepted (the builder only stores it)
msb_launch_config default_config(const msb_plan_s *, bool) {
    msb_launch_config c;
    std::memset(&c, 0, sizeof(c));
    c.rows_per_wg = 1;
    c.slots_fwd = c.slots_inv = 1;
    c.threads_x = c.threads_line = c.threads_tile = 256;
    c.lines_per_wg = c.lines_per_wave = 1;
    c.max_radix = 8;
    c.tile_run = 1;
    return c;
}
msb_status check_config(const msb_plan_s *, bool, const msb_launch_config &) { return MSB_OK; }
void solver_cache_free(msb_plan_s *) {}
void crack_free(msb_plan_s *) {}
}  // namespace msb
