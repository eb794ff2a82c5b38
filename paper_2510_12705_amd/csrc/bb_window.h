// bb_window.h -- device helpers shared by the stage kernels of both reductions
// (band -> bidiagonal in bb_kernels.hip, symmetric band -> tridiagonal in
// bb_sym.hip): the compute type of a storage type, global-address-space band
// pointers, raw buffer window accesses, agent-scope stores, the Householder update of one register-held
// segment, and the dependency poll.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "bb_device.h"

namespace bbk {

template <typename T>
struct Compute {
    using type = float;
};
template <>
struct Compute<double> {
    using type = double;
};

template <typename T>
__device__ __forceinline__ typename Compute<T>::type to_c(T x) {
    return static_cast<typename Compute<T>::type>(x);
}

// ---------------------------------------------------------------------------
// Addressing.  A lane's window base is the same for every thread of a wave (a
// wave never spans two lanes), so it is moved to scalar registers and every
// window access becomes scalar base + 32-bit lane offset (see buf_ld / buf_st).
// ---------------------------------------------------------------------------
// Other band pointers are kept in the global address space: generic (flat)
// accesses would also count against the LDS wait counter, so every LDS wait
// would wait for outstanding band loads as well.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;

template <typename T>
__device__ __forceinline__ gptr<T> to_global(T* p) { return (gptr<T>)(p); }

template <typename P>
__device__ __forceinline__ gptr<P> wave_uniform(P* ptr) {
    const uint64_t v = reinterpret_cast<uint64_t>(ptr);
    const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v >> 32));
    return reinterpret_cast<gptr<P>>((static_cast<uint64_t>(hi) << 32) | lo);
}

// a value known to be equal on every lane of the wave, moved to a scalar register
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }

// Window accesses go through raw buffer instructions: the
// descriptor holds the wave-uniform window base (scalar registers), each lane
// adds one 32-bit offset and a wave-uniform stride rides in the scalar offset,
// so a whole row or column segment needs one address register.  Offsets are in
// elements; the host keeps every in-window byte offset below 2^32, inside the
// descriptor's range.  Stores carry the agent-scope coherence bit (sc1), the
// same cache policy as st_agent.
using Rsrc = __amdgpu_buffer_rsrc_t;
constexpr int kBufDword3 = 0x00020000;  // gfx9 raw buffer: 32-bit data format, no swizzle
constexpr int kCpolSc1 = 16;            // cache-policy operand: sc1

template <typename T>
__device__ __forceinline__ Rsrc make_rsrc(gptr<T> base) {
    void* generic = reinterpret_cast<void*>(__builtin_bit_cast(uint64_t, base));
    return __builtin_amdgcn_make_buffer_rsrc(generic, (short)0, -1, kBufDword3);
}

template <typename T>
__device__ __forceinline__ T buf_ld(Rsrc r, int voff, int soff) {
    const int vb = (int)(static_cast<uint32_t>(voff) * static_cast<uint32_t>(sizeof(T)));
    const int sb = (int)(static_cast<uint32_t>(soff) * static_cast<uint32_t>(sizeof(T)));
    if constexpr (sizeof(T) == 8) {
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, vb, sb, 0));
    } else if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, vb, sb, 0));
    } else {
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b16(r, vb, sb, 0));
    }
}

template <typename T>
__device__ __forceinline__ void buf_st(Rsrc r, int voff, int soff, T v) {
    const int vb = (int)(static_cast<uint32_t>(voff) * static_cast<uint32_t>(sizeof(T)));
    const int sb = (int)(static_cast<uint32_t>(soff) * static_cast<uint32_t>(sizeof(T)));
    if constexpr (sizeof(T) == 8) {
        using V2 = __attribute__((ext_vector_type(2))) unsigned int;
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, v), r, vb, sb, kCpolSc1);
    } else if constexpr (sizeof(T) == 4) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, vb, sb, kCpolSc1);
    } else {
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, vb, sb, kCpolSc1);
    }
}

// Band stores are made at agent scope: each is coherent across the device once
// it is acknowledged, so a workgroup releases its results to another one by
// waiting for its stores (s_waitcnt) and then storing the progress word -- no
// write-back of the whole L2, which every agent-scope release fence would do.
template <typename T>
__device__ __forceinline__ void st_agent(gptr<T> p, T v) {
    if constexpr (sizeof(T) == 8) {
        __hip_atomic_store(reinterpret_cast<gptr<unsigned long long>>(p), __builtin_bit_cast(unsigned long long, v),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else if constexpr (sizeof(T) == 4) {
        __hip_atomic_store(reinterpret_cast<gptr<unsigned int>>(p), __builtin_bit_cast(unsigned int, v), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    } else {
        __hip_atomic_store(reinterpret_cast<gptr<unsigned short>>(p), __builtin_bit_cast(unsigned short, v),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// ---------------------------------------------------------------------------
// Householder application to one row / column segment of m+1 values held in
// registers: a <- a - (tau (a . v)) v.
//   FP64 storage: the dot is summed left to right with separate multiply and add
//   and the update is a - (tau w) v, i.e. the same IEEE operations as a plain
//   sequential implementation (no fused multiply-add; contraction is off).
//   FP32 / FP16 storage: single-precision arithmetic with compensated
//   accumulation.  The products are summed in blocks of kCompBlock by a chain
//   of fused multiply-adds, and the block sums are accumulated with TwoSum
//   (Knuth), whose rounding errors are summed separately and added at the end;
//   then a - fma(tau w, v).  Per term this costs about a quarter of the
//   instructions of compensating every product (Ogita-Rump-Oishi Dot2, the
//   earlier form), with the same measured accuracy.
// ---------------------------------------------------------------------------
template <typename C, int TWM>
__device__ __forceinline__ void apply_segment(C (&av)[TWM + 1], const C (&vs)[TWM + 1], C tau, int m) {
    if constexpr (std::is_same<C, double>::value) {
        // entries t > m are +0 in av and vs: they add exactly 0 and stay 0
        double w = 0.0;
#pragma unroll
        for (int t = 0; t <= TWM; ++t) w = w + av[t] * vs[t];
        const double tw = tau * w;
#pragma unroll
        for (int t = 0; t <= TWM; ++t) av[t] = av[t] - tw * vs[t];
    } else {
        constexpr int kCompBlock = 4;
        float s = 0.f, comp = 0.f;
#pragma unroll
        for (int g0 = 0; g0 <= TWM; g0 += kCompBlock) {
            float part = av[g0] * vs[g0];
#pragma unroll
            for (int t = g0 + 1; t < g0 + kCompBlock && t <= TWM; ++t) part = fmaf(av[t], vs[t], part);
            const float s1 = s + part;  // TwoSum(s, part) = s1 + es exactly
            const float bv = s1 - s;
            const float es = (s - (s1 - bv)) + (part - bv);
            s = s1;
            comp = comp + es;
        }
        const float tw = tau * (s + comp);
#pragma unroll
        for (int t = 0; t <= TWM; ++t) av[t] = fmaf(-tw, vs[t], av[t]);
    }
}

// Thread 0 only: spin until *flag >= need (or abort / watchdog).  Returns the value
// seen (>= need) or -1 on abort; ends with an agent-scope acquire (invalidates this
// CU's L1 and the stale lines of this XCD's L2).
__device__ __forceinline__ int poll_ge(const int* flag, int need, int* abort_flag, int* err_word, unsigned spin_limit) {
    unsigned spins = 0;
    int v;
    while ((v = __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) < need) {
        __builtin_amdgcn_s_sleep(1);
        if ((++spins & 255u) == 0) {
            if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return -1;
            if (spins > spin_limit) {
                __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(err_word, 2 /*BB_ERR_TIMEOUT*/, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                return -1;
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return v;
}

}  // namespace bbk
