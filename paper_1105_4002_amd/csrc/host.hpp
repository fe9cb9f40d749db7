// Host-side helpers shared by the C-ABI translation units: the geometry
// handle, error recording, device selection and workspace arithmetic.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <cmath>
#include <vector>

#include "tvreg.h"
#include "tvreg_internal.hpp"

// The opaque handle of the C ABI.
struct tvreg_geometry {
    tvreg_geometry_desc desc;
    std::vector<double> angles;
    std::vector<double> dirs;  // 3D parallel beam: 3 per view
    tvreg_precision prec;
    int device;
    tvr::GeomDev g;
    void *dev_tables;
    int64_t N, m;
    int pstride;  // partial-sum capacity per slot
    int sym_off;  // 1: a stored transpose ignores the scan's symmetry (tvreg_set_symmetry)
};

namespace tvr {

// Records the message returned by tvreg_last_error() and passes s through.
tvreg_status fail(tvreg_status s, const char *fmt, ...);
void clear_error();

// Argument checks shared by tvreg_solve and tvreg_solve_batched.
tvreg_status check_solve_params(const tvreg_solve_params *p);
// The feasible set the parameters select.
Box box_of(const tvreg_solve_params *p);

// The feasible set in storage type T: for float the bounds are rounded
// inward, so every stored iterate lies in Q (an empty result, lo > hi, means
// the box is narrower than one float).
template <typename T>
inline Box box_for(const tvreg_solve_params *p)
{
    Box b = box_of(p);
    if (sizeof(T) == sizeof(float)) {
        float lo = (float)b.lo, hi = (float)b.hi;
        if ((double)lo < b.lo)
            lo = nextafterf(lo, __builtin_inff());
        if ((double)hi > b.hi)
            hi = nextafterf(hi, -__builtin_inff());
        b.lo = lo;
        b.hi = hi;
    }
    return b;
}

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
inline size_t elem_size(tvreg_precision p) { return p == TVREG_F64 ? 8 : 4; }
inline size_t partial_bytes(int pstride) { return sizeof(double) * (size_t)S_COUNT * pstride; }

// Makes a device current for the duration of a call.
struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) {
            ok = false;
            return;
        }
        if (prev != dev && hipSetDevice(dev) != hipSuccess)
            ok = false;
    }
    ~DeviceGuard()
    {
        int cur;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev)
            (void)hipSetDevice(prev);
    }
};

// Waits for the work queued on st so far by polling an event from this
// thread (the solvers wait on the device after every line-search trial; a
// blocking wait adds the thread's wake-up latency to each of them).
inline hipError_t spin_sync(hipStream_t st, hipEvent_t ev)
{
    hipError_t e = hipEventRecord(ev, st);
    if (e != hipSuccess)
        return e;
    while ((e = hipEventQuery(ev)) == hipErrorNotReady) {
    }
    return e;
}

// Page-locked host slots of the scalar sums a solver reads after each
// line-search trial: the finaliser kernel writes them there directly (the
// memory is mapped for the device), and the host reads them once the event
// its reads wait on has completed.  p is null when the allocation failed.
struct HostScalars {
    double *p = nullptr;
    hipEvent_t done = nullptr;  // polled by spin_sync after each read
    HostScalars()
    {
        if (hipHostMalloc((void **)&p, sizeof(double) * S_COUNT, hipHostMallocDefault) !=
            hipSuccess)
            p = nullptr;
        if (p && hipEventCreateWithFlags(&done, hipEventDisableTiming) != hipSuccess) {
            (void)hipHostFree(p);
            p = nullptr;
            done = nullptr;
        }
    }
    ~HostScalars()
    {
        if (done)
            (void)hipEventDestroy(done);
        if (p)
            (void)hipHostFree(p);
    }
    HostScalars(const HostScalars &) = delete;
    HostScalars &operator=(const HostScalars &) = delete;
    double &operator[](int i) { return p[i]; }
    double operator[](int i) const { return p[i]; }
};

}  // namespace tvr

#define TVR_HIP(call)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return tvr::fail(TVREG_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));    \
    } while (0)

#define TVR_TRY(expr)                                                                          \
    do {                                                                                       \
        tvreg_status s_ = (expr);                                                              \
        if (s_ < 0)                                                                            \
            return s_;                                                                         \
    } while (0)
