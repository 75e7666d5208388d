// Named ranges on the host timeline for profilers (roctx ranges: rocprofv3 --marker-trace
// shows them around the library's calls).  The roctx library is opened at run time on first
// use; without it the ranges cost a branch and do nothing.
#pragma once

namespace hobi {

class TraceRange {
  public:
    explicit TraceRange(const char* name);
    ~TraceRange();
    TraceRange(const TraceRange&) = delete;
    TraceRange& operator=(const TraceRange&) = delete;

  private:
    bool on_ = false;
};

}  // namespace hobi
