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
// the result equals the sequential order bit for bit.  The entries that are
// already final one step earlier are loaded before that wait completes.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "bb_device.h"
#include "bb_internal.h"
#include "bb_window.h"

namespace bbk {

// Threads per workgroup NT: 512, or 256 for stages with b <= 64 (the left pass
// then fits 128 threads and the rows below the block 64), so that two sweeps
// fit a CU where the pipeline needs many sweeps in flight.

// LDS of one workgroup: the (TWM+1)^2 block (full square, compute type), one
// staging block of kWave columns of TWM+1 entries per wave of the left group,
// and a reflector scratch of 2 (TWM+1) doubles per wave.
template <typename C, int TWM, int NT>
struct SymLds {
    static constexpr int LDB = TWM + 1;
    static constexpr size_t block = 0;
    static constexpr size_t stage = (sizeof(C) * LDB * LDB + 15) / 16 * 16;
    static constexpr size_t scratch = stage + sizeof(C) * (NT == 512 ? 256 : 128) * LDB;
    static constexpr size_t scratch_per_wave = sizeof(double) * 2 * LDB;
    static constexpr size_t bytes = scratch + scratch_per_wave * (NT / kWave);
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

// One step of one sweep, executed by the whole workgroup.  Three parts touch
// disjoint entries and run at the same time in different waves: the left pass
// over the columns k+1 .. p-1 (rows p..p+m), the right pass over the rows below
// the block (p+m+1 .. L, columns p..p+m), and the block itself.  The left group
// (the first SymShape::kLeft threads) takes one column per thread, the right
// group (the following kRight threads) one row per thread (further items, for
// windows wider than a group, are loaded where they are used), and the last
// wave the block: its lanes 0..m apply the left pass to the block's columns,
// then, after a wave barrier, the right pass to its rows, each lane storing its
// row's part of the lower triangle.  Every global load of the step is issued at
// its start, the reflector column first (the reflector is formed while the
// others are in flight); the block's lower triangle is loaded by all threads
// and mirrored into LDS.
template <int NT>
struct SymShape {
    static constexpr int kLeft = NT == 512 ? 256 : 128;  // waves 0 .. kLeft/64 - 1
    static constexpr int kRight = NT - kLeft - kWave;    // then the right group
    static constexpr int kBlockWave = NT / kWave - 1;    // the last wave
};

template <typename T, int TWM, int NT, typename WaitFull>
__device__ __forceinline__ void sym_step(gptr<T> W, int64_t ldw, int n, int b, int k, int p, int m, int early_end,
                                         typename Compute<T>::type* blk, typename Compute<T>::type* stage,
                                         double* scr, WaitFull&& wait_full) {
    using C = typename Compute<T>::type;
    using Sh = SymShape<NT>;
    constexpr int LDB = TWM + 1;
    constexpr int NBE = (LDB * LDB + NT - 1) / NT;  // block entries per thread
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid / kWave;
    const bool left = tid < Sh::kLeft;
    const bool blockw = wave == Sh::kBlockWave;
    const bool right = !left && !blockw;
    const int gt = left ? tid : tid - Sh::kLeft;  // thread index within its group
    auto at = [&](int i, int q) { return W + ((int64_t)(i - q) + (int64_t)q * ldw); };
    const int nq = p - k - 1;                 // columns k+1 .. p-1 left of the block
    const int L = min(p + m + b, n - 1);
    const int nout = L - p - m;               // rows p+m+1 .. L below the block
    const int64_t rs = ldw - 1;               // stride of a row segment
    const int rs32 = (int)rs;
    // ---- loads ----
    const double xl = static_cast<double>(*at(p + min(lane, m), k));
    C a[TWM + 1];  // the left group's column, the right group's row, the block wave's column / row
    if (left && gt < nq) {
        const gptr<T> col = at(p, k + 1 + gt);
#pragma unroll
        for (int t = 0; t <= TWM; ++t) a[t] = to_c(col[min(t, m)]);
    }
    // rows below the block with p + m + 1 + gt < p + early_end are final before the full wait
    const bool row_early = right && gt < nout && m + 1 + gt < early_end;
    if (row_early) {
        const gptr<T> row = at(p + m + 1 + gt, p);
#pragma unroll
        for (int t = 0; t <= TWM; ++t) a[t] = to_c(row[(int64_t)min(t, m) * rs]);
    }
    C bv[NBE];
#pragma unroll
    for (int z = 0; z < NBE; ++z) {
        const int e = tid + z * NT;
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
        const int e = tid + z * NT;
        const int t = e / (m + 1), s = e - t * (m + 1);
        if (e < (m + 1) * (m + 1) && s >= t) {
            blk[s + t * LDB] = bv[z];
            blk[t + s * LDB] = bv[z];
        }
    }
    // A left-group wave's updated columns go through its LDS staging block and are
    // written back as contiguous runs (lane -> column u*CPI + lane/TWM, row lane%TWM
    // of store u; row TWM of every column in one more store), so the stores are
    // coalesced.
    C* wblk = stage + wave * (kWave * LDB);
    // A thread's first column or row, when loaded before the full wait, is also
    // updated before it (into the staging block, or kept in registers); only the
    // stores wait.
    const bool pre_left = left && gt < nq;
    if (pre_left || row_early) {
#pragma unroll
        for (int t = 0; t <= TWM; ++t) a[t] = t <= m ? a[t] : C(0);
        if (taud != 0.0) apply_segment<C, TWM>(a, vs, tau, m);
        if (pre_left) {
#pragma unroll
            for (int t = 0; t <= TWM; ++t) wblk[lane * LDB + t] = a[t];
        }
    }
    // the full dependency; it ends with a workgroup barrier, after which the rest is
    // loaded and every store is made
    if (!wait_full()) return;
    if (left) {
        // ---- left pass: one thread per column left of the block ----
        constexpr int CPI = kWave / TWM;
        const int sub = lane / TWM, tr = lane % TWM;
        for (int c0 = tid - lane; c0 < nq; c0 += Sh::kLeft) {  // the wave's first column
            const int ci = c0 + lane;
            if (ci < nq && ci != gt) {  // (the first column is in the staging block already)
                const gptr<T> col = at(p, k + 1 + ci);
#pragma unroll
                for (int t = 0; t <= TWM; ++t) a[t] = to_c(col[min(t, m)]);
#pragma unroll
                for (int t = 0; t <= TWM; ++t) a[t] = t <= m ? a[t] : C(0);
                if (taud != 0.0) apply_segment<C, TWM>(a, vs, tau, m);
#pragma unroll
                for (int t = 0; t <= TWM; ++t) wblk[lane * LDB + t] = a[t];
            }
            __builtin_amdgcn_wave_barrier();
            const int cmax = min(nq - c0, kWave);  // columns of this wave
            // column c0 + x starts x * rs elements after column c0
            const Rsrc base = make_rsrc(wave_uniform(at(p, k + 1 + c0)));
#pragma unroll
            for (int u = 0; u < TWM; ++u) a[u] = wblk[(u * CPI + sub) * LDB + tr];
            a[TWM] = wblk[lane * LDB + TWM];
            const int o = sub * rs32 + tr;
            // the stride is made opaque so that the per-store offsets are formed at the stores
            int step = CPI * rs32;
            asm volatile("" : "+s"(step));
#pragma unroll
            for (int u = 0; u < TWM; ++u)
                if (tr <= m && u * CPI + sub < cmax) buf_st<T>(base, o, u * step, static_cast<T>(a[u]));
            if (m == TWM && lane < cmax) buf_st<T>(base, lane * rs32, TWM, static_cast<T>(a[TWM]));
            __builtin_amdgcn_wave_barrier();  // the staging block is rewritten by the next iteration
        }
    } else if (right) {
        // ---- right pass below the block: one thread per row ----
        for (int ri = gt; ri < nout; ri += Sh::kRight) {
            const gptr<T> row = at(p + m + 1 + ri, p);  // A(p+m+1+ri, p+t) = row[t * rs]
            if (ri != gt || !row_early) {  // (an early first row is updated already)
#pragma unroll
                for (int t = 0; t <= TWM; ++t) a[t] = to_c(row[(int64_t)min(t, m) * rs]);
#pragma unroll
                for (int t = 0; t <= TWM; ++t) a[t] = t <= m ? a[t] : C(0);
                if (taud != 0.0) apply_segment<C, TWM>(a, vs, tau, m);
            }
#pragma unroll
            for (int t = 0; t <= TWM; ++t)
                if (t <= m) st_agent(row + (int64_t)t * rs, static_cast<T>(a[t]));
        }
    } else {
        // ---- the block: left pass on its columns, then right pass on its rows ----
        if (lane <= m) {
#pragma unroll
            for (int t = 0; t <= TWM; ++t) a[t] = t <= m ? blk[t + lane * LDB] : C(0);
            if (taud != 0.0) apply_segment<C, TWM>(a, vs, tau, m);
#pragma unroll
            for (int t = 0; t <= TWM; ++t)
                if (t <= m) blk[t + lane * LDB] = a[t];
        }
        __builtin_amdgcn_wave_barrier();
        if (lane <= m) {
            const int ri = lane;
#pragma unroll
            for (int t = 0; t <= TWM; ++t) a[t] = t <= m ? blk[ri + t * LDB] : C(0);
            if (taud != 0.0) apply_segment<C, TWM>(a, vs, tau, m);
#pragma unroll
            for (int t = 0; t <= TWM; ++t)
                if (t <= ri) st_agent(at(p + ri, p + t), static_cast<T>(a[t]));
            // column k becomes (beta, 0, ..., 0); every wave read its segment before the barrier
            st_agent(at(p + lane, k), static_cast<T>(lane == 0 ? betad : 0.0));
        }
    }
}

// One stage; progress[r] = steps completed by sweep r, kDone once it and every
// earlier sweep finished.
template <typename T, int TWM, int NT>
__global__ __launch_bounds__(NT, NT == 256 ? 2 : 1) void bb_sym_stage(SymStageArgs a) {
    using C = typename Compute<T>::type;
    extern __shared__ __align__(16) unsigned char smem[];
    using Lay = SymLds<C, TWM, NT>;
    C* blk = reinterpret_cast<C*>(smem + Lay::block);
    C* stg = reinterpret_cast<C*>(smem + Lay::stage);
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
        // Two-part wait.  Once sweep r-1 has completed one step less than the rule
        // asks, column k, the columns left of the block, the block and the rows
        // below it up to p + early_end - 1 are final (an exhaustive check of the
        // schedule shows it for every stage shape): they are loaded and the
        // reflector is formed first; the rest is loaded, and everything is stored,
        // after the full wait.
        const int early_end = c == 1 ? 2 * b - 1 : b - 1;
        for (int j = 0; j < len; ++j) {
            if (threadIdx.x == 0 && r > 0) {
                const int need = j + H - 1 > len_prev ? kDone : j + H - 1;
                if (need > known) {
                    const int v = poll_ge(a.progress + (r - 1), need, a.abort_flag, a.err_word, a.spin_limit);
                    if (v < 0) s_ok = 0;
                    else known = v;
                }
            }
            __syncthreads();
            if (!s_ok) return;
            auto wait_full = [&]() -> bool {  // every thread of the workgroup
                if (threadIdx.x == 0 && r > 0 && s_ok) {
                    const int need = j + H > len_prev ? kDone : j + H;
                    if (need > known) {
                        const int v = poll_ge(a.progress + (r - 1), need, a.abort_flag, a.err_word, a.spin_limit);
                        if (v < 0) s_ok = 0;
                        else known = v;
                    }
                }
                __syncthreads();
                return s_ok != 0;
            };
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
            sym_step<T, TWM, NT>(W, a.ldw, n, b, k, p, m, early_end, blk, stg, scr, wait_full);
            if (!s_ok) return;
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

template <typename T, int TWM, int NT>
static void launch_sym_twm(const SymStageArgs& a, int grid, hipStream_t st) {
    using C = typename Compute<T>::type;
    const size_t smem = SymLds<C, TWM, NT>::bytes;
    hipLaunchKernelGGL((bb_sym_stage<T, TWM, NT>), dim3(grid), dim3(NT), smem, st, a);
}

template <typename T, int TWM>
static void launch_sym_nt(const SymStageArgs& a, int nt, int grid, hipStream_t st) {
    if (nt == 256) launch_sym_twm<T, TWM, 256>(a, grid, st);
    else launch_sym_twm<T, TWM, 512>(a, grid, st);
}

template <typename T>
static hipError_t launch_sym_stage_t(const SymStageArgs& a, int twm, int nt, int grid, hipStream_t st) {
    switch (twm) {
        case 8: launch_sym_nt<T, 8>(a, nt, grid, st); break;
        case 16: launch_sym_nt<T, 16>(a, nt, grid, st); break;
        case 32: launch_sym_nt<T, 32>(a, nt, grid, st); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int sym_stage_threads(int b, int tw) {
    (void)tw;
    return b <= 64 ? 256 : 512;  // the 256-thread shape: 128 left-group and 64 right-group threads
}

hipError_t launch_sym_stage(int dtype, const SymStageArgs& a, int twm, int nt, int grid, hipStream_t st) {
    return dtype == 0 ? launch_sym_stage_t<double>(a, twm, nt, grid, st) : launch_sym_stage_t<float>(a, twm, nt, grid, st);
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
