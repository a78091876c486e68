// Kernel timing tracer: when enabled, every launch made through a ProfScope is
// bracketed by two HIP events recorded on the launch's stream.  Totals per
// kernel name are read back (after synchronising the events) as JSON.
#pragma once

#include <hip/hip_runtime.h>

namespace cta {

bool prof_enabled();
int prof_begin(const char* name, hipStream_t s);  // returns a record id or -1
void prof_end(int id, hipStream_t s);

struct ProfScope {
    int id;
    hipStream_t s;
    ProfScope(const char* name, hipStream_t st) : id(-1), s(st) {
        if (prof_enabled()) id = prof_begin(name, s);
    }
    ~ProfScope() {
        if (id >= 0) prof_end(id, s);
    }
};

}  // namespace cta
