// Launch statistics (HIP events around launches), see include/zolo_stats.h.
#pragma once

#include <hip/hip_runtime.h>

namespace zolo {

bool stats_on();
// Brackets one launch: construct before, call end() after the launch.
class StatScope {
  public:
    StatScope(const char* name, hipStream_t st, double flops, double bytes = 0.0);
    void end();

  private:
    int slot_ = -1;
    int pair_ = -1;
    hipStream_t st_ = nullptr;
};

}  // namespace zolo
