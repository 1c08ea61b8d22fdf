// apply_phi_noalloc.hip -- the fractional operator of Sec. 2.4 without a
// handle and without any device allocation (lbm_fade_apply_phi_noalloc in
// include/lbm_fade.h).
//
// The operator data (Toeplitz generator, boundary columns and BF16 splits of
// every axis, computed in FP64 on the host exactly as lbm_fade_create does)
// live in one fixed device array of the library.  Each device the library runs on holds its own copy
// of the array at its own address; the address is looked up once per device
// with hipGetSymbolAddress and only that pointer is handed to copies and
// kernels (the array's name in host code is not a device address).
#include "../../include/lbm_fade.h"

#include <hip/hip_runtime.h>
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

#include "lbm_handle.h"

namespace {

constexpr size_t kScratchBytes = size_t(16) << 20;  // LBM_NOALLOC_SCRATCH_BYTES
static_assert(kScratchBytes == LBM_NOALLOC_SCRATCH_BYTES, "header and library agree on the scratch size");
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mutex;
unsigned char* g_scratch_ptr[kMaxDevices] = {};

int fail(int code, const std::string& msg) { return lbm::set_error(code, msg.c_str()); }

// Device address of this device's copy of `scratch` (looked up on the first
// call with the device current, then kept).
int scratch_of(int dev, unsigned char** out)
{
    if (dev < 0 || dev >= kMaxDevices) return fail(LBM_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(LBM_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<unsigned char*>(p);
    }
    *out = g_scratch_ptr[dev];
    return LBM_OK;
}

}  // namespace

extern "C" int lbm_fade_apply_phi_noalloc(const lbm_grid* grid, const lbm_params* params, const float* C, float* Phi,
                                          void* stream)
{
    if (!grid || !params || !C || !Phi) return fail(LBM_EINVAL, "null argument");
    int rc = lbm::validate_config(grid, 2 * grid->dim + 1, params);
    if (rc) return rc;
    const int64_t nodes = (int64_t)grid->n[0] * grid->n[1] * (grid->dim == 3 ? grid->n[2] : 1);
    const size_t op_bytes = lbm::operator_image_bytes(*grid);
    const size_t need = op_bytes;
    if (need > kScratchBytes)
        return fail(LBM_EINVAL, "grid too large for the no-allocation entry point: needs " + std::to_string(need) +
                                    " bytes of its " + std::to_string(kScratchBytes) + "-byte device scratch");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(LBM_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return fail(LBM_EDEVICE, std::string("hipGetDeviceProperties: ") + hipGetErrorString(e));
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(LBM_EDEVICE, std::string("device is ") + prop.gcnArchName + ", this library is built for gfx950");
    unsigned char* base = nullptr;
    rc = scratch_of(dev, &base);
    if (rc) return rc;

    lbm::AxisOp ops[3];
    lbm::AxisLayout lays[3];
    std::vector<unsigned char> host(op_bytes, 0);
    lbm::build_operator_image(*grid, *params, host.data(), base, ops);
    lbm::make_layouts(*grid, lays);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // the host image is pageable memory freed on return: wait for the copy
    e = hipMemcpyAsync(base, host.data(), op_bytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(LBM_EDEVICE, std::string("upload of operator data: ") + hipGetErrorString(e));
    e = lbm::launch_fractional(ops, lays, grid->dim, params->precision, C, 0, Phi, nodes, s);
    if (e != hipSuccess) return fail(LBM_EDEVICE, std::string("fractional term: ") + hipGetErrorString(e));
    return LBM_OK;
}
