// roctx ranges through the ROCm profiler SDK's roctx library, looked up once at run time.
#include "trace.h"

#include <dlfcn.h>

#include <mutex>

namespace hobi {

namespace {

using PushFn = int (*)(const char*);
using PopFn = int (*)();

struct Roctx {
    PushFn push = nullptr;
    PopFn pop = nullptr;
};

const Roctx& roctx() {
    static Roctx r;
    static std::once_flag once;
    std::call_once(once, [] {
        const char* names[] = {"librocprofiler-sdk-roctx.so.1", "librocprofiler-sdk-roctx.so"};
        for (const char* n : names) {
            void* h = dlopen(n, RTLD_NOW | RTLD_LOCAL);
            if (!h) continue;
            PushFn push = (PushFn)dlsym(h, "roctxRangePushA");
            PopFn pop = (PopFn)dlsym(h, "roctxRangePop");
            if (push && pop) {
                r.push = push;
                r.pop = pop;
                return;
            }
        }
    });
    return r;
}

}  // namespace

TraceRange::TraceRange(const char* name) {
    const Roctx& r = roctx();
    if (r.push) {
        r.push(name);
        on_ = true;
    }
}

TraceRange::~TraceRange() {
    if (on_) roctx().pop();
}

}  // namespace hobi
