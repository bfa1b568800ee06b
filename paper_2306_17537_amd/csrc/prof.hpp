// Opt-in launch profiler: while enabled (ie_profile_begin .. ie_profile_end), every kernel
// launch of the operator and Krylov passes is bracketed by HIP events recorded on the stream it
// is launched on, together with the algorithmic bytes that launch must move (compulsory reads
// and writes of its inputs and outputs, counted once).  Disabled, a scope costs one branch.
#pragma once

#include <string>

#include "common.hpp"

namespace ie {

bool prof_enabled();
void prof_record(hipStream_t s, bool start, const std::string* key, double bytes);
// Launch groups: records made while a group is current can later have their bytes scaled
// (the fraction of batched problems that were still active when the launches ran).
long prof_new_group();
void prof_set_group(long g);  // -1: none
void prof_scale_group(long g, double scale);

struct ProfScope {
  hipStream_t s;
  bool on;
  ProfScope(hipStream_t st, const char* name, const char* tag, double bytes) : s(st), on(prof_enabled()) {
    if (on) {
      std::string key = std::string(name) + " " + tag;
      prof_record(s, true, &key, bytes);
    }
  }
  ~ProfScope() {
    if (on) prof_record(s, false, nullptr, 0);
  }
};

}  // namespace ie
