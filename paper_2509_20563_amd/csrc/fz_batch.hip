// Device side of batched calls: per-field result records, packing of the
// containers back to back (exclusive scan of their sizes on the device),
// and the header gather of a packed batch.
#include "fz_common.h"
#include "fz_kernels.h"

namespace fz {

// Compression record of one field: its staging slot, size and flags.
// Decompression record: flags, outlier codes met, regression blocks and
// the two outlier position hash sums.
__global__ void k_field_record(const Misc* misc, uint64_t slot, uint64_t* rec, int decode) {
    if (threadIdx.x != 0) return;
    if (decode) {
        rec[0] = misc->flags;
        rec[1] = misc->code0_count;
        rec[2] = misc->nreg;
        rec[3] = misc->ohash_dec;
        rec[4] = misc->ohash_list;
    } else {
        rec[0] = slot;
        rec[1] = misc->total_bytes;
        rec[2] = misc->flags;
    }
}

// offs[i] = sum over j < i of the 16-byte-rounded sizes (a failed field
// gets 0 bytes); offs[n] = total.  One workgroup, chunks of 1024 fields.
__global__ __launch_bounds__(1024) void k_pack_offsets(const uint64_t* __restrict__ rec, uint32_t n,
                                                       uint64_t* __restrict__ offs) {
    __shared__ uint64_t ws[16];
    __shared__ uint64_t carry;
    const uint32_t t = threadIdx.x, lane = t & 63, wave = t >> 6;
    if (t == 0) carry = 0;
    __syncthreads();
    for (uint32_t base = 0; base < n; base += 1024) {
        const uint32_t i = base + t;
        uint64_t v = 0;
        if (i < n) {
            const bool ok = (rec[3 * i + 2] & (F_NONFINITE | F_EB | F_INTERNAL | F_TIMEOUT)) == 0;
            v = ok ? (rec[3 * i + 1] + 15) & ~15ull : 0;
        }
        const uint64_t incl = wave_incl_scan64(v, [](uint64_t a, uint64_t b) { return a + b; });
        if (lane == 63) ws[wave] = incl;
        __syncthreads();
        uint64_t pre = carry;
        for (uint32_t w = 0; w < wave; w++) pre += ws[w];
        if (i < n) offs[i] = pre + incl - v;
        __syncthreads();
        if (t == 1023) carry = pre + incl;
        __syncthreads();
    }
    if (t == 0) offs[n] = carry;
}

// Copy each field's container from its staging slot to its packed offset;
// the bytes between its end and the next 16-byte boundary are zero.
__global__ __launch_bounds__(256) void k_pack_copy(const uint8_t* __restrict__ stage, const uint64_t* __restrict__ rec,
                                                   const uint64_t* __restrict__ offs, uint32_t n,
                                                   uint8_t* __restrict__ out) {
    const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint32_t f = 0; f < n; f++) {
        const uint64_t len = offs[f + 1] - offs[f];  // rounded size, 0 for a failed field
        const uint64_t size = rec[3 * f + 1];
        const uint4* src = reinterpret_cast<const uint4*>(stage + rec[3 * f]);
        uint4* dst = reinterpret_cast<uint4*>(out + offs[f]);
        for (uint64_t k = gid; k < len / 16; k += stride) {
            uint4 v = src[k];
            if (16 * k + 16 > size) {
                // the last, partial chunk
                uint8_t b[16];
                __builtin_memcpy(b, &v, 16);
                for (int j = 0; j < 16; j++)
                    if (16 * k + j >= size) b[j] = 0;
                __builtin_memcpy(&v, b, 16);
            }
            dst[k] = v;
        }
    }
}

// Headers of a packed batch (offs on the device) -> hdr[128 n].
__global__ __launch_bounds__(256) void k_gather_headers(const uint8_t* __restrict__ in, const uint64_t* __restrict__ offs,
                                                        uint32_t n, uint8_t* __restrict__ hdr) {
    const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t k = gid; k < (uint64_t)n * (kHdr / 16); k += stride) {
        const uint64_t f = k / (kHdr / 16), j = k % (kHdr / 16);
        reinterpret_cast<uint4*>(hdr)[k] = reinterpret_cast<const uint4*>(in + offs[f])[j];
    }
}

void launch_field_record(hipStream_t st, const Misc* misc, uint64_t slot, uint64_t* rec, int decode) {
    hipLaunchKernelGGL(k_field_record, dim3(1), dim3(64), 0, st, misc, slot, rec, decode);
}

void launch_pack(hipStream_t st, const uint8_t* stage, const uint64_t* rec, uint64_t* offs, uint32_t n, uint8_t* out) {
    hipLaunchKernelGGL(k_pack_offsets, dim3(1), dim3(1024), 0, st, rec, n, offs);
    hipLaunchKernelGGL(k_pack_copy, dim3(2048), dim3(256), 0, st, stage, rec, offs, n, out);
}

void launch_gather_headers(hipStream_t st, const uint8_t* in, const uint64_t* offs, uint32_t n, uint8_t* hdr) {
    uint64_t grid = ((uint64_t)n * (kHdr / 16) + 255) / 256;
    if (grid > 1024) grid = 1024;
    hipLaunchKernelGGL(k_gather_headers, dim3((uint32_t)grid), dim3(256), 0, st, in, offs, n, hdr);
}

}  // namespace fz
