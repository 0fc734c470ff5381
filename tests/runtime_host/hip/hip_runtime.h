// CPU stand-in of the HIP host API the library's runtime and server use, for running their
// host code under sanitizers in tests (never part of the library).  Every stream has a
// worker thread that executes its operations later, in order, so asynchronous copies read
// and write host buffers when a GPU would, events complete when the stream reaches them,
// and several streams run at once.  Stream capture records the operations of the capturing
// stream (and of streams that join it through an event) into a graph that a launch replays.
// "Device" memory is host memory.
#pragma once

#include <atomic>
#include <condition_variable>
#include <cstddef>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <memory>
#include <mutex>
#include <set>
#include <thread>
#include <vector>

// device-side keywords and built-ins that the shared headers mention (never executed here)
#define __device__
#define __host__
#define __global__
#define __forceinline__ inline
struct dim3 {
    unsigned x, y, z;
    dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct fh_block_index {
    unsigned x = 0, y = 0, z = 0;
};
inline fh_block_index blockIdx;

struct float2 {
    float x, y;
};
inline float2 make_float2(float a, float b) { return float2{a, b}; }

typedef int hipError_t;
enum {
    hipSuccess = 0,
    hipErrorInvalidValue = 1,
    hipErrorNotReady = 600,
    hipErrorOutOfMemory = 2,
};
enum hipMemcpyKind {
    hipMemcpyHostToDevice = 1,
    hipMemcpyDeviceToHost = 2,
    hipMemcpyDeviceToDevice = 3,
};
enum { hipStreamNonBlocking = 1, hipEventDisableTiming = 2, hipHostMallocDefault = 0 };
enum hipStreamCaptureMode { hipStreamCaptureModeThreadLocal = 1 };
enum { hipMemoryTypeHost = 0, hipMemoryTypeDevice = 1, hipMemoryTypeManaged = 2 };
struct hipPointerAttribute_t {
    int type;
};

namespace fakehip {

using Op = std::function<void()>;

struct Graph {
    std::vector<Op> ops;
    std::shared_ptr<std::atomic<bool>> alive = std::make_shared<std::atomic<bool>>(true);
};

struct Stream;

struct Event {
    std::mutex m;
    std::condition_variable cv;
    uint64_t recorded = 0;    // generation of the last record
    uint64_t reached = 0;     // generation the stream has reached
    std::atomic<Graph*> capture{nullptr}; // recorded during capture into this graph
};

struct Stream {
    std::mutex m;
    std::condition_variable cv, idle;
    std::deque<Op> q;
    bool busy = false, stop = false;
    std::atomic<Graph*> capture{nullptr};  // capturing into
    std::thread th;
    Stream() {
        th = std::thread([this] {
            std::unique_lock<std::mutex> lk(m);
            for (;;) {
                cv.wait(lk, [&] { return stop || !q.empty(); });
                if (q.empty() && stop) return;
                Op op = std::move(q.front());
                q.pop_front();
                busy = true;
                lk.unlock();
                op();
                lk.lock();
                busy = false;
                if (q.empty()) idle.notify_all();
            }
        });
    }
    void push(Op op) {
        if (Graph* g = capture.load()) {
            g->ops.push_back(std::move(op));
            return;
        }
        std::lock_guard<std::mutex> lk(m);
        q.push_back(std::move(op));
        cv.notify_one();
    }
    void drain() {
        std::unique_lock<std::mutex> lk(m);
        idle.wait(lk, [&] { return q.empty() && !busy; });
    }
    ~Stream() {
        {
            std::lock_guard<std::mutex> lk(m);
            stop = true;
        }
        cv.notify_all();
        th.join();
    }
};

struct Registry {
    std::mutex m;
    std::set<Stream*> streams;
    std::set<const void*> device;
    std::vector<std::pair<const char*, size_t>> ranges;
    static Registry& get() {
        static Registry r;
        return r;
    }
    bool on_device(const void* p) {
        std::lock_guard<std::mutex> lk(m);
        for (auto& r : ranges)
            if ((const char*)p >= r.first && (const char*)p < r.first + r.second) return true;
        return false;
    }
    void device_sync() {
        std::vector<Stream*> all;
        {
            std::lock_guard<std::mutex> lk(m);
            all.assign(streams.begin(), streams.end());
        }
        for (Stream* s : all) s->drain();
    }
};

// The default stream: a stream of its own (the library only uses non-blocking streams).
inline Stream* null_stream() {
    static Stream* s = [] {
        auto* n = new Stream();
        std::lock_guard<std::mutex> lk(Registry::get().m);
        Registry::get().streams.insert(n);
        return n;
    }();
    return s;
}

}  // namespace fakehip

typedef fakehip::Stream* hipStream_t;
typedef fakehip::Event* hipEvent_t;
typedef fakehip::Graph* hipGraph_t;
typedef fakehip::Graph* hipGraphExec_t;

inline fakehip::Stream* fh_stream(hipStream_t s) { return s ? s : fakehip::null_stream(); }

inline hipError_t hipGetLastError() { return hipSuccess; }
inline const char* hipGetErrorString(hipError_t) { return "stand-in error"; }
inline hipError_t hipSetDevice(int) { return hipSuccess; }
inline hipError_t hipGetDevice(int* d) {
    *d = 0;
    return hipSuccess;
}
inline hipError_t hipGetDeviceCount(int* n) {
    *n = 1;
    return hipSuccess;
}
inline hipError_t hipMemGetInfo(size_t* f, size_t* t) {
    *f = (size_t)1 << 34;
    *t = *f;
    return hipSuccess;
}

inline hipError_t hipMalloc(void** p, size_t n) {
    *p = std::malloc(n);
    if (!*p) return hipErrorOutOfMemory;
    auto& r = fakehip::Registry::get();
    std::lock_guard<std::mutex> lk(r.m);
    r.ranges.push_back({(const char*)*p, n});
    return hipSuccess;
}
inline hipError_t hipFree(void* p) {
    auto& r = fakehip::Registry::get();
    r.device_sync();                         // hipFree synchronizes the device
    {
        std::lock_guard<std::mutex> lk(r.m);
        for (size_t i = 0; i < r.ranges.size(); ++i)
            if (r.ranges[i].first == p) {
                r.ranges.erase(r.ranges.begin() + i);
                break;
            }
    }
    std::free(p);
    return hipSuccess;
}
inline hipError_t hipHostMalloc(void** p, size_t n, unsigned) {
    *p = std::malloc(n);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}
inline hipError_t hipHostFree(void* p) {
    std::free(p);
    return hipSuccess;
}
inline hipError_t hipPointerGetAttributes(hipPointerAttribute_t* a, const void* p) {
    a->type = fakehip::Registry::get().on_device(p) ? hipMemoryTypeDevice : hipMemoryTypeHost;
    return hipSuccess;
}

inline hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
    *s = new fakehip::Stream();
    auto& r = fakehip::Registry::get();
    std::lock_guard<std::mutex> lk(r.m);
    r.streams.insert(*s);
    return hipSuccess;
}
inline hipError_t hipStreamDestroy(hipStream_t s) {
    s->drain();
    {
        auto& r = fakehip::Registry::get();
        std::lock_guard<std::mutex> lk(r.m);
        r.streams.erase(s);
    }
    delete s;
    return hipSuccess;
}
inline hipError_t hipStreamSynchronize(hipStream_t s) {
    if (fh_stream(s)->capture) std::abort();     // not allowed while capturing
    fh_stream(s)->drain();
    return hipSuccess;
}

inline hipError_t hipMemcpyAsync(void* d, const void* src, size_t n, hipMemcpyKind, hipStream_t s) {
    fh_stream(s)->push([=] { std::memcpy(d, src, n); });
    return hipSuccess;
}
inline hipError_t hipMemcpy(void* d, const void* src, size_t n, hipMemcpyKind) {
    fakehip::Registry::get().device_sync();
    std::memcpy(d, src, n);
    return hipSuccess;
}
inline hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t s) {
    fh_stream(s)->push([=] { std::memset(d, v, n); });
    return hipSuccess;
}

inline hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) {
    *e = new fakehip::Event();
    return hipSuccess;
}
inline hipError_t hipEventCreate(hipEvent_t* e) { return hipEventCreateWithFlags(e, 0); }
inline hipError_t hipEventDestroy(hipEvent_t e) {
    delete e;
    return hipSuccess;
}
inline hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
    fakehip::Stream* st = fh_stream(s);
    if (fakehip::Graph* cg = st->capture.load()) {
        e->capture = cg;
        return hipSuccess;
    }
    uint64_t g;
    {
        std::lock_guard<std::mutex> lk(e->m);
        e->capture = nullptr;
        g = ++e->recorded;
    }
    st->push([e, g] {
        std::lock_guard<std::mutex> lk(e->m);
        if (e->reached < g) e->reached = g;
        e->cv.notify_all();
    });
    return hipSuccess;
}
inline hipError_t hipEventQuery(hipEvent_t e) {
    std::lock_guard<std::mutex> lk(e->m);
    return e->reached >= e->recorded ? hipSuccess : hipErrorNotReady;
}
inline hipError_t hipEventSynchronize(hipEvent_t e) {
    std::unique_lock<std::mutex> lk(e->m);
    e->cv.wait(lk, [&] { return e->reached >= e->recorded; });
    return hipSuccess;
}
inline hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) {
    *ms = 0.01f;
    return hipSuccess;
}
inline hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned) {
    fakehip::Stream* st = fh_stream(s);
    if (fakehip::Graph* g = e->capture.load()) {     // joins the capture of the recording stream
        st->capture = g;
        return hipSuccess;
    }
    if (st->capture) return hipSuccess;     // inside the graph the order is already serial
    uint64_t g;
    {
        std::lock_guard<std::mutex> lk(e->m);
        g = e->recorded;
    }
    st->push([e, g] {
        std::unique_lock<std::mutex> lk(e->m);
        e->cv.wait(lk, [&] { return e->reached >= g; });
    });
    return hipSuccess;
}

inline hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
    if (fh_stream(s)->capture) std::abort();
    fh_stream(s)->capture = new fakehip::Graph();
    return hipSuccess;
}
inline hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g) {
    fakehip::Stream* st = fh_stream(s);
    *g = st->capture.load();
    auto& r = fakehip::Registry::get();
    std::lock_guard<std::mutex> lk(r.m);
    for (fakehip::Stream* o : r.streams) {
        fakehip::Graph* mine = *g;
        o->capture.compare_exchange_strong(mine, nullptr);   // joined streams leave the capture
    }
    st->capture = nullptr;
    return hipSuccess;
}
inline hipError_t hipGraphInstantiate(hipGraphExec_t* ex, hipGraph_t g, void*, void*, size_t) {
    *ex = new fakehip::Graph();
    (*ex)->ops = g->ops;
    return hipSuccess;
}
// A launched graph's operations check that its executable still exists when they run.
inline hipError_t hipGraphLaunch(hipGraphExec_t ex, hipStream_t s) {
    auto alive = ex->alive;
    for (auto& op : ex->ops)
        fh_stream(s)->push([op, alive] {
            if (!*alive) std::abort();
            op();
        });
    return hipSuccess;
}
inline hipError_t hipGraphExecDestroy(hipGraphExec_t ex) {
    *ex->alive = false;
    delete ex;
    return hipSuccess;
}
inline hipError_t hipGraphDestroy(hipGraph_t g) {
    delete g;
    return hipSuccess;
}
