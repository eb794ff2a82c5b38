// bb_sym.hip -- symmetric band -> tridiagonal reduction on gfx950.
//
// The bulge chase of the bidiagonal reduction, for a symmetric matrix held as
// its lower band: the same stages of successive band reduction (inner
// tilewidth TW) and the same step geometry, but one reflector per step, applied
// from both sides (A <- H A H).  Step (k, p, m) of a sweep:
//   reflector from the column segment A[p..p+m, k] (column k becomes beta, 0..0);
//   left pass: rows p..p+m of columns k+1 .. p-1, and the whole (m+1)^2 diagonal
//              block (its upper triangle is the mirror of the stored lower one);
//   right pass: columns p..p+m of the block's rows and of rows p+m+1 .. L,
//              L = min(p+m+b, n-1);
//   the block's lower triangle is stored back.
// Working band (lower layout): A(i, q) = W[(i - q) + q * ldw] for 0 <= i - q < ldw,
// ldw >= b + TW + 2 (room for the bulge fill below the band).  A column segment
// is contiguous; a row segment has stride ldw - 1.
//
// Scheduling: one persistent workgroup per sweep at a time (sweeps claimed in
// order); step j of sweep r waits until sweep r-1 has completed j + H steps or is
// done, with H = 2 for c >= 2 and 3 for c = 1 (the smallest lag for which steps
// left unordered touch disjoint entries; checked exhaustively on the CPU).  So
// the result equals the sequential order bit for bit.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "bb_device.h"
#include "bb_internal.h"
#include "bb_window.h"

namespace bbk {

constexpr int kSymThreads = 256;

// LDS of one workgroup: the (TWM+1)^2 block (full square, compute type) and a
// reflector scratch of 2 (TWM+1) doubles per wave.
template <typename C, int TWM>
struct SymLds {
    static constexpr int LDB = TWM + 1;
    static constexpr size_t block = 0;
    static constexpr size_t scratch = (sizeof(C) * LDB * LDB + 15) / 16 * 16;
    static constexpr size_t scratch_per_wave = sizeof(double) * 2 * LDB;
    static constexpr size_t bytes = scratch + scratch_per_wave * (kSymThreads / kWave);
};

template <typename T>
__global__ void bb_sym_pack(const T* __restrict__ band, int64_t ldband, int64_t n, int64_t b, T* __restrict__ W,
                            int64_t ldw) {
    const int64_t total = n * ldw;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t q = idx / ldw, o = idx - q * ldw;  // row q + o of column q
        W[idx] = (o <= b && q + o < n) ? band[o + q * ldband] : T(0);
    }
}

template <typename T>
__global__ void bb_sym_extract(const T* __restrict__ W, int64_t n, int64_t ldw, double* __restrict__ d,
                               double* __restrict__ e) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        d[i] = static_cast<double>(W[i * ldw]);
        if (i + 1 < n) e[i] = static_cast<double>(W[1 + i * ldw]);
    }
}

// One step of one sweep, executed by the whole workgroup.  Every global load of
// the step is issued at its start, the reflector column first (so the reflector
// is formed while the others are in flight): thread `tid` holds the column
// k+1+tid of the left pass and the row p+tid of the right pass (further items,
// for windows wider than the workgroup, are loaded where they are used), and
// the block's lower triangle is loaded into registers and mirrored into LDS.
template <typename T, int TWM>
__device__ __forceinline__ void sym_step(gptr<T> W, int64_t ldw, int n, int b, int k, int p, int m,
                                         typename Compute<T>::type* blk, double* scr) {
    using C = typename Compute<T>::type;
    constexpr int LDB = TWM + 1;
    constexpr int NBE = (LDB * LDB + kSymThreads - 1) / kSymThreads;  // block entries per thread
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    auto at = [&](int i, int q) { return W + ((int64_t)(i - q) + (int64_t)q * ldw); };
    const int nq = p - k - 1;                 // columns k+1 .. p-1 left of the block
    const int L = min(p + m + b, n - 1);
    const int nrows = L - p + 1;              // rows p .. L of the right pass
    const int64_t rs = ldw - 1;               // stride of a row segment
    // ---- loads ----
    const double xl = static_cast<double>(*at(p + min(lane, m), k));
    C aL[TWM + 1], aR[TWM + 1];
    if (tid < nq) {
        const gptr<T> col = at(p, k + 1 + tid);
#pragma unroll
        for (int t = 0; t <= TWM; ++t) aL[t] = to_c(col[min(t, m)]);
    }
    if (tid > m && tid < nrows) {
        const gptr<T> row = at(p + tid, p);
#pragma unroll
        for (int t = 0; t <= TWM; ++t) aR[t] = to_c(row[(int64_t)min(t, m) * rs]);
    }
    C bv[NBE];
#pragma unroll
    for (int z = 0; z < NBE; ++z) {
        const int e = tid + z * kSymThreads;
        const int t = e / (m + 1), s = e - t * (m + 1);
        bv[z] = (e < (m + 1) * (m + 1) && s >= t) ? to_c(*at(p + s, p + t)) : C(0);
    }
    // ---- reflector (every wave; FP64 for every storage type) ----
    C vs[TWM + 1];
    double taud, betad, v_own, v_hi;
    house_lds<TWM>(xl, 0.0, m, scr, vs, taud, betad, v_own, v_hi);
    const C tau = static_cast<C>(taud);
    // ---- the block, mirrored to a full square: blk[s + t * LDB] = A(p+s, p+t) ----
#pragma unroll
    for (int z = 0; z < NBE; ++z) {
        const int e = tid + z * kSymThreads;
        const int t = e / (m + 1), s = e - t * (m + 1);
        if (e < (m + 1) * (m + 1) && s >= t) {
            blk[s + t * LDB] = bv[z];
            blk[t + s * LDB] = bv[z];
        }
    }
    __syncthreads();
    // ---- left pass: one thread per column ----
    for (int ci = tid; ci < nq + m + 1; ci += kSymThreads) {
        if (ci < nq) {
            const gptr<T> col = at(p, k + 1 + ci);
            if (ci != tid) {
#pragma unroll
                for (int t = 0; t <= TWM; ++t) aL[t] = to_c(col[min(t, m)]);
            }
#pragma unroll
            for (int t = 0; t <= TWM; ++t) aL[t] = t <= m ? aL[t] : C(0);
            if (taud != 0.0) apply_segment<C, TWM>(aL, vs, tau, m);
#pragma unroll
            for (int t = 0; t <= TWM; ++t)
                if (t <= m) st_agent(col + t, static_cast<T>(aL[t]));
        } else {
            const int t2 = ci - nq;
            C av[TWM + 1];
#pragma unroll
            for (int t = 0; t <= TWM; ++t) av[t] = t <= m ? blk[t + t2 * LDB] : C(0);
            if (taud != 0.0) apply_segment<C, TWM>(av, vs, tau, m);
#pragma unroll
            for (int t = 0; t <= TWM; ++t)
                if (t <= m) blk[t + t2 * LDB] = av[t];
        }
    }
    __syncthreads();
    // ---- right pass: one thread per row (the block's rows, then rows p+m+1 .. L) ----
    for (int ri = tid; ri < nrows; ri += kSymThreads) {
        if (ri <= m) {
            C av[TWM + 1];
#pragma unroll
            for (int t = 0; t <= TWM; ++t) av[t] = t <= m ? blk[ri + t * LDB] : C(0);
            if (taud != 0.0) apply_segment<C, TWM>(av, vs, tau, m);
#pragma unroll
            for (int t = 0; t <= TWM; ++t)
                if (t <= m) blk[ri + t * LDB] = av[t];
        } else {
            const gptr<T> row = at(p + ri, p);  // A(p + ri, p + t) = row[t * rs]
            if (ri != tid) {
#pragma unroll
                for (int t = 0; t <= TWM; ++t) aR[t] = to_c(row[(int64_t)min(t, m) * rs]);
            }
#pragma unroll
            for (int t = 0; t <= TWM; ++t) aR[t] = t <= m ? aR[t] : C(0);
            if (taud != 0.0) apply_segment<C, TWM>(aR, vs, tau, m);
#pragma unroll
            for (int t = 0; t <= TWM; ++t)
                if (t <= m) st_agent(row + (int64_t)t * rs, static_cast<T>(aR[t]));
        }
    }
    __syncthreads();
    // ---- the block's lower triangle goes back; column k becomes (beta, 0, ..., 0) ----
#pragma unroll
    for (int z = 0; z < NBE; ++z) {
        const int e = tid + z * kSymThreads;
        const int t = e / (m + 1), s = e - t * (m + 1);
        if (e < (m + 1) * (m + 1) && s >= t) st_agent(at(p + s, p + t), static_cast<T>(blk[s + t * LDB]));
    }
    if (tid <= m) st_agent(at(p + tid, k), static_cast<T>(tid == 0 ? betad : 0.0));
}

// One stage; progress[r] = steps completed by sweep r, kDone once it and every
// earlier sweep finished.
template <typename T, int TWM>
__global__ __launch_bounds__(kSymThreads) void bb_sym_stage(SymStageArgs a) {
    using C = typename Compute<T>::type;
    extern __shared__ __align__(16) unsigned char smem[];
    using Lay = SymLds<C, TWM>;
    C* blk = reinterpret_cast<C*>(smem + Lay::block);
    double* scr = reinterpret_cast<double*>(smem + Lay::scratch + Lay::scratch_per_wave * (threadIdx.x / kWave));
    __shared__ int s_r, s_ok;
    const gptr<T> W = to_global(reinterpret_cast<T*>(a.W));
    const int n = a.n, b = a.b, tw = a.tw, c = a.c, H = a.H;
    auto steps_of = [&](int r) { return 1 + (n - 2 - r - c) / b; };  // steps of sweep r (r <= n - c - 2)
    for (;;) {
        if (threadIdx.x == 0) {
            int r = atomicAdd(a.claim, 1);
            if (__hip_atomic_load(a.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) r = a.nsweeps;
            s_r = r;
            s_ok = 1;
        }
        __syncthreads();
        const int r = s_r;
        if (r >= a.nsweeps) return;
        const int len = steps_of(r);
        const int len_prev = r > 0 ? steps_of(r - 1) : 0;
        int known = 0;
        for (int j = 0; j < len; ++j) {
            if (threadIdx.x == 0 && r > 0) {
                const int need = j + H > len_prev ? kDone : j + H;
                if (need > known) {
                    const int v = poll_ge(a.progress + (r - 1), need, a.abort_flag, a.err_word, a.spin_limit);
                    if (v < 0) s_ok = 0;
                    else known = v;
                }
            }
            __syncthreads();
            if (!s_ok) return;
            int k, p, m;
            if (j == 0) {
                k = r;
                p = r + c;
                m = min(r + b, n - 1) - p;
            } else {
                k = r + c + (j - 1) * b;
                p = k + b;
                m = min(tw, n - 1 - p);
            }
            sym_step<T, TWM>(W, a.ldw, n, b, k, p, m, blk, scr);
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();  // every wave's agent-scope stores are complete
            if (threadIdx.x == 0)
                __hip_atomic_store(a.progress + r, j + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (threadIdx.x == 0) {
            int ok = 1;
            if (r > 0 && known < kDone &&
                poll_ge(a.progress + (r - 1), kDone, a.abort_flag, a.err_word, a.spin_limit) < 0)
                ok = 0;
            if (ok) __hip_atomic_store(a.progress + r, kDone, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s_ok = ok;
        }
        __syncthreads();
        if (!s_ok) return;
    }
}

template <typename T, int TWM>
static void launch_sym_twm(const SymStageArgs& a, int grid, hipStream_t st) {
    using C = typename Compute<T>::type;
    const size_t smem = SymLds<C, TWM>::bytes;
    hipLaunchKernelGGL((bb_sym_stage<T, TWM>), dim3(grid), dim3(kSymThreads), smem, st, a);
}

template <typename T>
static hipError_t launch_sym_stage_t(const SymStageArgs& a, int twm, int grid, hipStream_t st) {
    switch (twm) {
        case 8: launch_sym_twm<T, 8>(a, grid, st); break;
        case 16: launch_sym_twm<T, 16>(a, grid, st); break;
        case 32: launch_sym_twm<T, 32>(a, grid, st); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_sym_stage(int dtype, const SymStageArgs& a, int twm, int grid, hipStream_t st) {
    return dtype == 0 ? launch_sym_stage_t<double>(a, twm, grid, st) : launch_sym_stage_t<float>(a, twm, grid, st);
}

hipError_t launch_sym_pack(int dtype, const void* band, int64_t ldband, int64_t n, int64_t b, void* W, int64_t ldw,
                           hipStream_t st) {
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((n * ldw + 255) / 256, 65536));
    if (dtype == 0)
        hipLaunchKernelGGL(bb_sym_pack<double>, dim3(grid), dim3(256), 0, st, static_cast<const double*>(band), ldband,
                           n, b, static_cast<double*>(W), ldw);
    else
        hipLaunchKernelGGL(bb_sym_pack<float>, dim3(grid), dim3(256), 0, st, static_cast<const float*>(band), ldband,
                           n, b, static_cast<float*>(W), ldw);
    return hipGetLastError();
}

hipError_t launch_sym_extract(int dtype, const void* W, int64_t n, int64_t ldw, double* d, double* e, hipStream_t st) {
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 65536));
    if (dtype == 0)
        hipLaunchKernelGGL(bb_sym_extract<double>, dim3(grid), dim3(256), 0, st, static_cast<const double*>(W), n, ldw,
                           d, e);
    else
        hipLaunchKernelGGL(bb_sym_extract<float>, dim3(grid), dim3(256), 0, st, static_cast<const float*>(W), n, ldw,
                           d, e);
    return hipGetLastError();
}

}  // namespace bbk
