// Host stand-ins for the few HIP runtime calls that the library's host-only
// sources (layout, device cache, worker pool) make, so that those sources
// build and run on a CPU under the sanitizers.  "Device" memory is host
// memory from malloc; there is one device, 0, per thread.
#include <hip/hip_runtime_api.h>

#include <cstdlib>

namespace {
thread_local int tl_device = 0;
}

extern "C" {

hipError_t hipGetDevice(int* deviceId) {
    if (!deviceId) return hipErrorInvalidValue;
    *deviceId = tl_device;
    return hipSuccess;
}

hipError_t hipSetDevice(int deviceId) {
    if (deviceId != 0) return hipErrorInvalidDevice;
    tl_device = deviceId;
    return hipSuccess;
}

hipError_t hipMalloc(void** ptr, size_t size) {
    if (!ptr) return hipErrorInvalidValue;
    *ptr = std::malloc(size ? size : 1);
    return *ptr ? hipSuccess : hipErrorOutOfMemory;
}

hipError_t hipFree(void* ptr) {
    std::free(ptr);
    return hipSuccess;
}

hipError_t hipGetLastError(void) { return hipSuccess; }

}  // extern "C"
