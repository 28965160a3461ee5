// Library-owned device scratch, one buffer per device, reused across calls
// (see cbct_internal.h).  A call takes the device's buffer under a lock,
// makes its stream wait for the previous user's completion event, enqueues
// its work and records the event again before releasing the lock, so calls
// on different streams never overlap on the buffer.  The buffer grows (once,
// after the previous user has finished) when a call needs more.
#include <hip/hip_runtime.h>

#include <mutex>

#include "cbct_internal.h"

namespace cbct {
namespace {

constexpr int kMaxDevices = 64;

struct DevScratch {
    void *ptr = nullptr;
    size_t bytes = 0;
    hipEvent_t last = nullptr;   // completion of the latest user's work
};

std::mutex g_mutex[kMaxDevices];
DevScratch g_scratch[kMaxDevices];

}  // namespace

hipError_t scratch_acquire(size_t bytes, hipStream_t s, ScratchLease &lease)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    if (dev < 0 || dev >= kMaxDevices)
        return hipErrorInvalidDevice;
    lease.lock = std::unique_lock<std::mutex>(g_mutex[dev]);
    lease.device = dev;
    DevScratch &S = g_scratch[dev];
    if (!S.last) {
        e = hipEventCreateWithFlags(&S.last, hipEventDisableTiming);
        if (e != hipSuccess)
            return e;
    } else {
        e = hipStreamWaitEvent(s, S.last, 0);
        if (e != hipSuccess)
            return e;
    }
    if (S.bytes < bytes) {
        if (S.ptr) {
            e = hipEventSynchronize(S.last);
            if (e != hipSuccess)
                return e;
            e = hipFree(S.ptr);
            S.ptr = nullptr;
            S.bytes = 0;
            if (e != hipSuccess)
                return e;
        }
        e = hipMalloc(&S.ptr, bytes);
        if (e != hipSuccess) {
            S.ptr = nullptr;
            return e;
        }
        S.bytes = bytes;
    }
    lease.ptr = S.ptr;
    return hipSuccess;
}

hipError_t scratch_release(hipStream_t s, ScratchLease &lease)
{
    hipError_t e = hipSuccess;
    if (lease.device >= 0 && g_scratch[lease.device].last)
        e = hipEventRecord(g_scratch[lease.device].last, s);
    lease.ptr = nullptr;
    lease.device = -1;
    if (lease.lock.owns_lock())
        lease.lock.unlock();
    return e;
}

}  // namespace cbct
