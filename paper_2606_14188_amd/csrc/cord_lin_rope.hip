// Instantiations of the banded direct linearization for rope size classes.
#include "cord_kernels.h"
#include "cord_lin_direct.h"

namespace cord {

hipError_t linearize_rope_direct(int nmax, const KArgs& a, int nblk, int tmax, hipStream_t s, bool* handled) {
    *handled = false;
    static int lds_max = -1;
    if (lds_max < 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
            v = 0;
        lds_max = v;
    }
    size_t need = 0;
    hipError_t (*fn)(const KArgs&, int, int, hipStream_t) = nullptr;
    switch (nmax) {
    case 32: fn = &LinDirect<128, 32, kMaxObs>::launch; need = LinDirect<128, 32, kMaxObs>::kLds; break;
    case 64: fn = &LinDirect<192, 64, kMaxObs>::launch; need = LinDirect<192, 64, kMaxObs>::kLds; break;
    case 128: fn = &LinDirect<384, 128, kMaxObs>::launch; need = LinDirect<384, 128, kMaxObs>::kLds; break;
    default: return hipSuccess;
    }
    if ((size_t)lds_max < need) return hipSuccess;
    *handled = true;
    return fn(a, nblk, tmax, s);
}

}  // namespace cord
