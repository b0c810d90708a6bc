// Entry point that allocates nothing: the stable key-value radix sort of
// sph_sort_kv (Sec. 3.1; the stable order of the worked example of Sec. 4.3)
// with its scratch in a fixed device array of this file instead of a
// context's buffers, for callers that cannot allocate device memory.
#include <mutex>

#include "sph_internal.h"

namespace {

constexpr uint32_t kNoAllocMaxN = 1u << 21;  // keys per call, at most
constexpr uint32_t kNoAllocTiles = (kNoAllocMaxN + sph::kSortTile - 1) / sph::kSortTile;
// one ping-pong pair (keys, values), the per-tile digit counts, the digit totals
constexpr size_t kNoAllocKeysOff = 0;
constexpr size_t kNoAllocValsOff = kNoAllocKeysOff + (size_t)kNoAllocMaxN * 4;
constexpr size_t kNoAllocHistOff = kNoAllocValsOff + (size_t)kNoAllocMaxN * 4;
constexpr size_t kNoAllocTotOff = kNoAllocHistOff + (size_t)256 * kNoAllocTiles * 4;
constexpr size_t kNoAllocBytes = kNoAllocTotOff + 256 * 4;

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch_dev[kMaxDevices];  // the array's address on each device, once looked up

}  // namespace

// Each GPU the library runs on holds its own copy of this array until the
// process ends. In host code the name is only a stand-in for the symbol: the
// device address comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

// The device address of `scratch` on the current device, looked up once per
// device (with that device current); nullptr and a message on failure.
void *scratch_on(int dev, std::string *err) {
    if (dev < 0 || dev >= kMaxDevices) {
        *err = "device index out of range for the fixed scratch table";
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            *err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            return nullptr;
        }
        g_scratch_dev[dev] = ptr;
    }
    return g_scratch_dev[dev];
}

}  // namespace

extern "C" int sph_sort_kv_noalloc(const uint32_t *keys, const int32_t *vals, uint32_t *keys_out,
                                   int32_t *vals_out, uint32_t n, int key_bits, void *stream) {
    if (key_bits < 1 || key_bits > 32)
        return sph::set_error(SPH_E_INVALID_ARG, "sph_sort_kv_noalloc: key_bits must be 1..32");
    if (n > kNoAllocMaxN)
        return sph::set_error(SPH_E_CAPACITY,
                              "sph_sort_kv_noalloc: n = %u exceeds the fixed scratch of %u keys", n,
                              kNoAllocMaxN);
    if (n == 0) return SPH_OK;
    if (!keys || !vals || !keys_out || !vals_out)
        return sph::set_error(SPH_E_INVALID_ARG, "sph_sort_kv_noalloc: null array");
    if ((const void *)keys == (const void *)keys_out || (const void *)vals == (const void *)vals_out)
        return sph::set_error(SPH_E_INVALID_ARG, "sph_sort_kv_noalloc: outputs must not alias inputs");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return sph::set_error(SPH_E_HIP, "sph_sort_kv_noalloc: hipGetDevice: %s", hipGetErrorString(e));
    std::string err;
    unsigned char *base = (unsigned char *)scratch_on(dev, &err);
    if (!base) return sph::set_error(SPH_E_HIP, "sph_sort_kv_noalloc: %s", err.c_str());
    e = sph::radix_sort_bufs(keys, vals, keys_out, vals_out, n, key_bits,
                             (uint32_t *)(base + kNoAllocKeysOff), (int32_t *)(base + kNoAllocValsOff),
                             (uint32_t *)(base + kNoAllocHistOff), (uint32_t *)(base + kNoAllocTotOff),
                             (hipStream_t)stream);
    if (e != hipSuccess)
        return sph::set_error(SPH_E_HIP, "sph_sort_kv_noalloc: %s", hipGetErrorString(e));
    return SPH_OK;
}
