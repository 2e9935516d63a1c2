// Registry of the instantiated 2-D MMA sweep kernels and the device shape
// their launches use.
#include <hip/hip_runtime.h>

#include "mma2d_impl.hpp"

namespace ss {

hipError_t device_shape(int *cus, int *xcds) {
    constexpr int kMaxDevices = 64;
    static int cache[kMaxDevices][2];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    if (cache[dev][0] == 0) {
        int c = 0, x = 0;
        if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipDeviceGetAttribute(&x, hipDeviceAttributeNumberOfXccs, dev) != hipSuccess || c < 1)
            return hipErrorInvalidDevice;
        cache[dev][1] = x > 0 ? x : 1;
        cache[dev][0] = c;
    }
    *cus = cache[dev][0];
    *xcds = cache[dev][1];
    return hipSuccess;
}

namespace {

bool same_key(const MmaKey &a, const MmaKey &b) {
    return a.r1 == b.r1 && a.r2 == b.r2 && a.kc == b.kc && a.rad == b.rad && a.mode == b.mode &&
           a.part == b.part && a.state == b.state;
}

template <class F>
void for_each_entry(F f) {
    const MmaEntry *(*tables[])(int *) = {mma_table_f32_r1, mma_table_f32_r2, mma_table_f32_r3, mma_table_f16,
                                          mma_table_planes, mma_table_planes3};
    for (auto table : tables) {
        int n = 0;
        const MmaEntry *t = table(&n);
        for (int i = 0; i < n; ++i) f(t[i]);
    }
}

}  // namespace

MmaLaunch find_mma2d(const MmaKey &k) {
    MmaLaunch fn = nullptr;
    for_each_entry([&](const MmaEntry &e) {
        if (!fn && same_key(e.key, k)) fn = e.fn;
    });
    return fn;
}

bool mma2d_geometry(const MmaKey &k, int *wgh, int *row, int *pw, int *padg) {
    bool found = false;
    for_each_entry([&](const MmaEntry &e) {
        if (!found && same_key(e.key, k)) {
            *wgh = e.wgh;
            *row = e.row;
            *pw = e.pw;
            *padg = e.padg;
            found = true;
        }
    });
    return found;
}

int mma2d_keys(int rad, int mode, int part, int state, MmaKey *out, int max) {
    int n = 0;
    for_each_entry([&](const MmaEntry &e) {
        if (e.key.rad == rad && e.key.mode == mode && e.key.part == part && e.key.state == state && n < max)
            out[n++] = e.key;
    });
    return n;
}

}  // namespace ss
