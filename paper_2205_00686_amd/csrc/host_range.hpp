// A named range in the profiler's marker trace (rocprofv3 --marker-trace) around a host entry point
// that enqueues or waits for device work.  Without a profiler attached the calls return at once.
#pragma once
#include <rocprofiler-sdk-roctx/roctx.h>

namespace lbm {
struct HostRange {
  explicit HostRange(const char* name) { roctxRangePushA(name); }
  ~HostRange() { roctxRangePop(); }
  HostRange(const HostRange&) = delete;
  HostRange& operator=(const HostRange&) = delete;
};
}  // namespace lbm
