// Failure injection for tests of the error paths: a countdown per kind of
// failure point; when it reaches zero that point fails once (a host
// allocation throws std::bad_alloc, a device allocation reports
// hipErrorOutOfMemory, a HIP launch step reports hipErrorLaunchFailure).
// Off (countdown < 0) unless a test arms it through ustat_debug_inject.
#pragma once

#include <cstdint>
#include <new>

namespace ustat {

enum InjectKind : int32_t { INJ_HOST_ALLOC = 0, INJ_DEVICE_ALLOC = 1, INJ_HIP = 2, INJ_KINDS = 3 };

// Arm kind `kind`: the (countdown + 1)-th point of that kind reached from
// now fails; a negative countdown disarms it.
void inject_arm(int kind, int64_t countdown);
// Called at a failure point: true exactly when this point must fail.
bool inject_fire(int kind);

// A host allocation failure point.
inline void inject_host_alloc() {
    if (inject_fire(INJ_HOST_ALLOC)) throw std::bad_alloc();
}

}  // namespace ustat
