// Rates of the units the dense vote uses, measured on the current device:
// LDS atomic adds (conflict free, and with the bank pattern of lane groups
// voting random bins), 32-bit integer VALU, packed 16-bit integer VALU, and
// an HBM copy.  Each kernel repeats one kind of instruction in a loop; the
// rate is the work it issues over its duration (events around the launch,
// best of several launches).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "internal.h"

namespace sas {
void set_error(const std::string &msg);
}

namespace {

constexpr int kThreads = 512;
constexpr int kHistWords = 8192;  // 32 KB of LDS per workgroup
constexpr int kAddrs = 16;        // addresses per lane, reused in every round

// pattern 0: every wave adds to 64 consecutive words (two passes over the 32
// banks, no conflict).  pattern 1: the lanes form 4 groups of 16; each group
// adds to the 16 consecutive words of one random bin (the lane-group vote
// pattern), so groups that share a half-wave may meet in a bank.
__global__ void __launch_bounds__(kThreads) k_lds_atomic(uint32_t *out, int rounds, int pattern) {
    __shared__ uint32_t h[kHistWords];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int i = tid; i < kHistWords; i += kThreads) h[i] = 0;
    uint32_t addr[kAddrs];
#pragma unroll
    for (int u = 0; u < kAddrs; ++u) {
        if (pattern == 0) {
            addr[u] = (uint32_t)(wave * 1024 + ((u * 64 + lane) & 1023));
        } else {
            const uint32_t g = (uint32_t)(lane >> 4), j = (uint32_t)(lane & 15);
            uint32_t hsh = (uint32_t)(blockIdx.x * 131 + wave * 17 + u) * 0x9E3779B1u ^
                           (g * 0x85EBCA77u + 0x27d4eb2fu);
            hsh ^= hsh >> 15;
            hsh *= 0x2c1b3c6du;
            hsh ^= hsh >> 12;
            addr[u] = (hsh % (kHistWords / 16)) * 16 + j;
        }
    }
    __syncthreads();
    for (int r = 0; r < rounds; ++r) {
#pragma unroll
        for (int u = 0; u < kAddrs; ++u)
            __hip_atomic_fetch_add(&h[addr[u]], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    __syncthreads();
    if (tid < 64) out[blockIdx.x * 64 + tid] = h[tid * 128 + blockIdx.x % 128];
}

// Eight independent chains of (add, xor) per lane: 16 integer ops a round.
__global__ void __launch_bounds__(kThreads) k_valu_int32(uint32_t *out, int rounds) {
    uint32_t a[8];
    const uint32_t t = blockIdx.x * kThreads + threadIdx.x;
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = t * (k + 3);
    const uint32_t c1 = t | 1u, c2 = t ^ 0x5bd1e995u;
    for (int r = 0; r < rounds; ++r) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            asm volatile("v_add_u32 %0, %0, %1" : "+v"(a[k]) : "v"(c1));
            asm volatile("v_xor_b32 %0, %0, %1" : "+v"(a[k]) : "v"(c2));
        }
    }
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) s ^= a[k];
    out[t] = s;
}

// The same with packed 16-bit halves: 32 half-ops a round.
__global__ void __launch_bounds__(kThreads) k_valu_int16x2(uint32_t *out, int rounds) {
    uint32_t a[8];
    const uint32_t t = blockIdx.x * kThreads + threadIdx.x;
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = t * (k + 5);
    const uint32_t c1 = t | 0x10001u, c2 = t ^ 0x3c6ef372u;
    for (int r = 0; r < rounds; ++r) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            asm volatile("v_pk_add_u16 %0, %0, %1" : "+v"(a[k]) : "v"(c1));
            asm volatile("v_pk_sub_u16 %0, %0, %1" : "+v"(a[k]) : "v"(c2));
        }
    }
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) s ^= a[k];
    out[t] = s;
}

__global__ void __launch_bounds__(256) k_copy(const uint4 *__restrict__ src,
                                              uint4 *__restrict__ dst, int64_t n4) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride)
        dst[i] = src[i];
}

sas_status cfail(hipError_t e, const char *what) {
    sas::set_error(std::string("sas_measure_ceilings: ") + what + ": " + hipGetErrorString(e));
    return SAS_E_DEVICE;
}

}  // namespace

extern "C" sas_status sas_measure_ceilings(sas_ceilings *out, void *stream) {
    if (!out) {
        sas::set_error("sas_measure_ceilings: null output");
        return SAS_E_INVALID;
    }
    hipStream_t s = (hipStream_t)stream;
    int dev = 0, n_cu = 256;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return cfail(e, "device");
    hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    const int blocks = n_cu * 4;  // resident workgroups of 512 threads at 32 KB of LDS
    const int64_t copy_bytes = (int64_t)1 << 30;
    void *buf = nullptr, *src = nullptr, *dst = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    sas_status st = SAS_OK;
    auto best_of = [&](auto launch, int reps, float *ms_best) -> hipError_t {
        *ms_best = 1e30f;
        for (int r = 0; r < reps; ++r) {
            hipError_t he = hipEventRecord(ev[0], s);
            if (he != hipSuccess) return he;
            launch();
            if ((he = hipGetLastError()) != hipSuccess) return he;
            if ((he = hipEventRecord(ev[1], s)) != hipSuccess) return he;
            if ((he = hipEventSynchronize(ev[1])) != hipSuccess) return he;
            float ms = 0.f;
            if ((he = hipEventElapsedTime(&ms, ev[0], ev[1])) != hipSuccess) return he;
            *ms_best = std::min(*ms_best, ms);
        }
        return hipSuccess;
    };
    do {
        if ((e = hipEventCreate(&ev[0])) != hipSuccess || (e = hipEventCreate(&ev[1])) != hipSuccess) {
            st = cfail(e, "events");
            break;
        }
        if ((e = hipMalloc(&buf, (size_t)blocks * kThreads * sizeof(uint32_t))) != hipSuccess) {
            st = cfail(e, "allocation");
            break;
        }
        uint32_t *o = (uint32_t *)buf;
        const int lds_rounds = 2048;
        float ms = 0.f;
        for (int pattern = 0; pattern < 2; ++pattern) {
            e = best_of([&] {
                hipLaunchKernelGGL(k_lds_atomic, dim3(blocks), dim3(kThreads), 0, s, o, lds_rounds,
                                   pattern);
            }, 3, &ms);
            if (e != hipSuccess) break;
            const double lane_atomics = (double)blocks * kThreads * kAddrs * lds_rounds;
            (pattern == 0 ? out->lds_atomic_conflict_free : out->lds_atomic_lane_groups) =
                lane_atomics / (ms * 1e-3);
        }
        if (e != hipSuccess) {
            st = cfail(e, "LDS atomics");
            break;
        }
        const int valu_rounds = 4096;
        e = best_of([&] {
            hipLaunchKernelGGL(k_valu_int32, dim3(blocks), dim3(kThreads), 0, s, o, valu_rounds);
        }, 3, &ms);
        if (e != hipSuccess) {
            st = cfail(e, "int32 VALU");
            break;
        }
        out->valu_int32_ops = (double)blocks * kThreads * 16.0 * valu_rounds / (ms * 1e-3);
        e = best_of([&] {
            hipLaunchKernelGGL(k_valu_int16x2, dim3(blocks), dim3(kThreads), 0, s, o, valu_rounds);
        }, 3, &ms);
        if (e != hipSuccess) {
            st = cfail(e, "int16x2 VALU");
            break;
        }
        out->valu_int16x2_ops = (double)blocks * kThreads * 32.0 * valu_rounds / (ms * 1e-3);
        if ((e = hipMalloc(&src, copy_bytes)) != hipSuccess ||
            (e = hipMalloc(&dst, copy_bytes)) != hipSuccess ||
            (e = hipMemsetAsync(src, 1, copy_bytes, s)) != hipSuccess) {
            st = cfail(e, "copy buffers");
            break;
        }
        const int64_t n4 = copy_bytes / 16;
        e = best_of([&] {
            hipLaunchKernelGGL(k_copy, dim3(n_cu * 16), dim3(256), 0, s, (const uint4 *)src,
                               (uint4 *)dst, n4);
        }, 5, &ms);
        if (e != hipSuccess) {
            st = cfail(e, "HBM copy");
            break;
        }
        out->hbm_copy_bytes_per_s = 2.0 * (double)copy_bytes / (ms * 1e-3);
    } while (false);
    if (src) (void)hipFree(src);
    if (dst) (void)hipFree(dst);
    if (buf) (void)hipFree(buf);
    for (hipEvent_t v : ev)
        if (v) (void)hipEventDestroy(v);
    return st;
}
