// Instantiations of the banded direct linearization for rope size classes.
#include <atomic>

#include "cord_kernels.h"
#include "cord_lin_direct.h"

namespace cord {

namespace {

struct DirectClass {
    size_t lds = 0, slot = 0;
    int (*resident)() = nullptr;
    hipError_t (*launch)(const KArgs&, int, int, hipStream_t) = nullptr;
};

bool direct_class(int nmax, DirectClass* c) {
    switch (nmax) {
    case 32:
        *c = {LinDirect<128, 32, kMaxObs>::kLds, LinDirect<128, 32, kMaxObs>::kSlot,
              &LinDirect<128, 32, kMaxObs>::resident_per_cu, &LinDirect<128, 32, kMaxObs>::launch};
        return true;
    case 64:
        *c = {LinDirect<192, 64, kMaxObs>::kLds, LinDirect<192, 64, kMaxObs>::kSlot,
              &LinDirect<192, 64, kMaxObs>::resident_per_cu, &LinDirect<192, 64, kMaxObs>::launch};
        return true;
    case 128:
        *c = {LinDirect<384, 128, kMaxObs>::kLds, LinDirect<384, 128, kMaxObs>::kSlot,
              &LinDirect<384, 128, kMaxObs>::resident_per_cu, &LinDirect<384, 128, kMaxObs>::launch};
        return true;
    default:
        return false;
    }
}

// Workgroups of class nmax a CU keeps resident (0: the class cannot run,
// its LDS does not fit).  Queried once per class.
int per_cu(int nmax, const DirectClass& c) {
    static std::atomic<int> cap[3] = {-1, -1, -1};
    const int k = nmax == 32 ? 0 : nmax == 64 ? 1 : 2;
    if (cap[k].load() < 0) {
        int dev = 0, lds_max = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
            lds_max = 0;
        cap[k].store(((size_t)lds_max < c.lds) ? 0 : c.resident());
    }
    return cap[k].load();
}

}  // namespace

size_t linearize_rope_direct_scratch(int nmax, int* wg_per_cu) {
    *wg_per_cu = 0;
    DirectClass c;
    if (!direct_class(nmax, &c)) return 0;
    const int r = per_cu(nmax, c);
    if (r < 1) return 0;
    *wg_per_cu = r;
    return (size_t)kept_slots(r) * c.slot + kept_guard_floats(r);
}

hipError_t linearize_rope_direct(int nmax, const KArgs& a, int nblk, int tmax, hipStream_t s) {
    DirectClass c;
    if (!direct_class(nmax, &c)) return hipErrorInvalidValue;
    return c.launch(a, nblk, tmax, s);
}

}  // namespace cord
