// kmg_normals_static: kmg_normals without a workspace argument, for callers
// that cannot allocate device memory.  Its scratch (the cell hash table, the
// cell-sorted points, degrees and status of the radius search) lives in one
// file-scope device array per GPU, sized for kStaticMaxPoints kept points.
//
// The array's name is a host-side stand-in in host code: its device address
// is looked up once per device with hipGetSymbolAddress (on the first call
// made with that device current) and only that address is passed on.  Every
// call on a device shares the array and leaves its contents behind; the
// kernels clear what they need cleared themselves, so overlapping calls on one
// device race and must be serialised by the caller.
#include <mutex>

#include "kmg_internal.h"

namespace {

constexpr int64_t kStaticMaxPoints = KMG_STATIC_MAX_POINTS;
constexpr size_t kStaticScratchBytes = size_t(20) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (nullptr if it cannot be had).
void* scratch_of_current_device() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        g_ptr[dev] = p;
    }
    return g_ptr[dev];
}

}  // namespace

extern "C" __attribute__((visibility("default"))) kmg_status kmg_normals_static(
    const float* xyz, int64_t m, const kmg_params* p, float* normals, uint8_t* flags, int32_t* nbr_off,
    int32_t* nbr_idx, int64_t nbr_cap, int64_t* nnz, int32_t* n_normal, void* stream) {
    if (!p || !nnz || m < 0 || nbr_cap < 0 || !nbr_off) return KMG_ERR_ARG;
    if (p->mode != KMG_MODE_FASTER_PFH) return KMG_ERR_ARG;  // the classic mode keeps extra lists in scratch
    if (m > kStaticMaxPoints) return KMG_ERR_RANGE;
    if (kmg::normals_ws(m, KMG_MODE_FASTER_PFH, 0) > kStaticScratchBytes) return KMG_ERR_RANGE;
    void* ws = scratch_of_current_device();
    if (!ws) return KMG_ERR_DEVICE;
    return kmg_normals(xyz, m, p, normals, flags, nbr_off, nbr_idx, nbr_cap, nnz, n_normal, ws, kStaticScratchBytes,
                       stream);
}
