// Named host-side phase ranges for the profiler's marker trace
// (rocprofv3 --marker-trace): a context's creation and its parts (label scan
// and plan, sweep autotuning, modal set-up), the recording of a step graph,
// each advance, a gradient and its forward and reverse passes, a batch's
// creation, recording and advance.  The ranges time the host side of a call;
// device work they enqueue shows in the kernel trace inside them, and calls
// that synchronise (creation, gradients) cover their device work as well.
// A push/pop pair costs well under a microsecond when no profiler listens.
#pragma once

#include <rocprofiler-sdk-roctx/roctx.h>

namespace expint {

// Open from construction until end() or destruction, whichever comes first.
class PhaseRange {
 public:
  explicit PhaseRange(const char* name) { roctxRangePushA(name); }
  ~PhaseRange() { end(); }
  void end() {
    if (open_) roctxRangePop();
    open_ = false;
  }
  PhaseRange(const PhaseRange&) = delete;
  PhaseRange& operator=(const PhaseRange&) = delete;

 private:
  bool open_ = true;
};

}  // namespace expint
