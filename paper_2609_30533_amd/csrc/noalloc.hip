// noalloc.hip -- st_check_edges_noalloc: the discretised edge check of
// st_check_edges with its work lists in a fixed device array instead of
// buffers the library allocates, for callers that cannot allocate (code under
// HIP graph capture, tight serving loops).
//
// The edge pipeline's scratch (state counts, least-hit indices, rank lists of
// work items and their counters) lives in the file-scope array `scratch`.
// Host code never passes the array's name to a kernel: the name is a host
// stand-in, not a device address.  The first call on a device, with that
// device current, asks the runtime for the array's device address and keeps
// it per device; every later launch uses that address.  Each device holds its
// own copy of the array until the process ends, and every call on a device
// shares it: two calls that overlap on one device race.  The rank counters,
// which must start at zero, are cleared by a small fill kernel at the start of
// every call (no memset node, so the call can be captured into a graph).
#include <mutex>

#include "pipeline.hpp"
#include "st_internal.hpp"

namespace st {

constexpr int64_t kNoAllocMaxEdges = ST_NOALLOC_MAX_EDGES;
constexpr int kNoAllocItems = 16;  // work items per edge at most (the rank lists)
constexpr int kNoAllocCounters = kNoAllocItems * kCntStride;

// byte offsets of the sections (each a multiple of 256)
constexpr size_t kOffN = 0;
constexpr size_t kOffHit = kOffN + (size_t)kNoAllocMaxEdges * sizeof(int32_t);
constexpr size_t kOffItems = kOffHit + (size_t)kNoAllocMaxEdges * sizeof(int32_t);
constexpr size_t kOffCnt = kOffItems + (size_t)kNoAllocMaxEdges * kNoAllocItems * sizeof(int2);
constexpr size_t kScratchBytes = kOffCnt + (size_t)kNoAllocCounters * sizeof(int32_t);
static_assert(kOffHit % 256 == 0 && kOffItems % 256 == 0 && kOffCnt % 256 == 0, "section alignment");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static void *g_scratch_ptr[kMaxDevices];
static std::mutex g_scratch_mu;

// The device address of `scratch` on the current device (looked up once per
// device); null with the error set on failure.
static unsigned char *scratch_on_current_device() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        set_error("st_check_edges_noalloc: no current HIP device");
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            set_error("st_check_edges_noalloc: hipGetSymbolAddress failed: %s", hipGetErrorString(e));
            return nullptr;
        }
        g_scratch_ptr[dev] = ptr;
    }
    return (unsigned char *)g_scratch_ptr[dev];
}

__global__ void k_zero_i32(int32_t *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

}  // namespace st

using namespace st;

extern "C" int st_check_edges_noalloc(st_problem *p, int64_t E, const float *xa, const float *xb,
                                      uint8_t *free_out, int32_t *first_hit, void *stream) {
    if (!p || E < 0 || (E > 0 && (!xa || !xb || !free_out))) {
        set_error("st_check_edges_noalloc: bad arguments");
        return ST_EINVAL;
    }
    if (E > kNoAllocMaxEdges) {
        set_error("st_check_edges_noalloc: %lld edges exceed the fixed work area of %lld edges",
                  (long long)E, (long long)kNoAllocMaxEdges);
        return ST_EINVAL;
    }
    if (E == 0) return ST_OK;
    unsigned char *base = scratch_on_current_device();
    if (!base) return ST_EHIP;
    EdgeBufs eb;
    eb.cap = kNoAllocMaxEdges;
    eb.mmax = kNoAllocItems;
    eb.n = (int32_t *)(base + kOffN);
    eb.hit = (int32_t *)(base + kOffHit);
    eb.items = (int2 *)(base + kOffItems);
    eb.cnt = (int32_t *)(base + kOffCnt);
    const hipStream_t s = (hipStream_t)stream;
    k_zero_i32<<<(kNoAllocCounters + 255) / 256, 256, 0, s>>>(eb.cnt, kNoAllocCounters);
    ST_HIP(hipGetLastError());
    ST_HIP(launch_check_edges(p->sc, eb, E, xa, xb, nullptr, free_out, first_hit, p->tune_api, s, nullptr,
                              split_for(p->split_api, E)));
    return ST_OK;
}
