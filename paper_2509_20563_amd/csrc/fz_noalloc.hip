// Allocation-free decompression (fz_decompress_noalloc): the scratch of a
// first-order Lorenzo decode lives in one statically sized device array,
// which every GPU the library runs on holds until the process ends.  Its
// device address is taken once per device with hipGetSymbolAddress; host
// code uses that address only (the array's name is a host-side stand-in).
#include <mutex>

#include "../../include/fz.h"
#include "fz_common.h"
#include "fz_kernels.h"

using namespace fz;

namespace {

constexpr uint32_t kNoAllocBlocks = FZ_NOALLOC_MAX_BLOCKS;
constexpr int kMaxDevices = 64;

constexpr uint64_t up256(uint64_t v) { return (v + 255) & ~255ull; }

// Layout of the scratch array (each part 256-byte aligned).
constexpr uint64_t kOffMisc = 0;
constexpr uint64_t kOffHist = up256(kOffMisc + sizeof(Misc));
constexpr uint64_t kOffLut = up256(kOffHist + sizeof(uint32_t) * kHistCopies * kBins);
// look-back descriptors of the chunk scan: one per 1024 blocks, and more
// than enough for the scan's tiles of max_blocks blocks
constexpr uint64_t kDescEntries = kNoAllocBlocks / 1024 + 64;
constexpr uint64_t kOffDesc = up256(kOffLut + sizeof(uint16_t) * kLut);
constexpr uint64_t kOffOff = up256(kOffDesc + sizeof(uint64_t) * kDescEntries);
constexpr uint64_t kOffOidx = up256(kOffOff + sizeof(uint64_t) * kNoAllocBlocks);
constexpr uint64_t kScratchBytes = up256(kOffOidx + sizeof(uint2) * kNoAllocBlocks);

static __device__ __align__(256) uint8_t scratch[kScratchBytes];

struct DevScratch {
    std::once_flag once;
    int rc = FZ_OK;
    uint8_t* ptr = nullptr;
};
DevScratch g_dev[kMaxDevices];

// The device address of this device's scratch array (first call on a
// device: hipGetSymbolAddress with that device current).
int scratch_of(int dev, uint8_t** out) {
    if (dev < 0 || dev >= kMaxDevices) return FZ_ERR_ARG;
    DevScratch& d = g_dev[dev];
    std::call_once(d.once, [&] {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            hipGetLastError();
            d.rc = FZ_ERR_HIP;
            return;
        }
        d.ptr = (uint8_t*)p;
    });
    *out = d.ptr;
    return d.rc;
}

}  // namespace

extern "C" {

uint64_t fz_noalloc_scratch_bytes(void) { return kScratchBytes; }

int fz_decompress_noalloc(const void* d_in, uint64_t in_bytes, const void* h_hdr, float* d_out, uint64_t out_elems,
                          void* stream) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return FZ_ERR_HIP;
    uint8_t* base = nullptr;
    int rc = scratch_of(dev, &base);
    if (rc) return rc;
    DecodeScratch s;
    s.misc = reinterpret_cast<Misc*>(base + kOffMisc);
    s.hist = reinterpret_cast<uint32_t*>(base + kOffHist);
    s.lut = reinterpret_cast<uint16_t*>(base + kOffLut);
    s.desc_chunks = reinterpret_cast<uint64_t*>(base + kOffDesc);
    s.off = reinterpret_cast<uint64_t*>(base + kOffOff);
    s.oidx = reinterpret_cast<uint2*>(base + kOffOidx);
    s.max_blocks = kNoAllocBlocks;
    if (scan_tiles(kNoAllocBlocks) > kDescEntries) return FZ_ERR_INTERNAL;
    return decompress_on_scratch(s, d_in, in_bytes, h_hdr, d_out, out_elems, (hipStream_t)stream);
}

}  // extern "C"
