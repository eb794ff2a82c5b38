// bb_kernels.hip -- gfx950 kernels of the band -> bidiagonal reduction.
//
//   bb_pack     LAPACK upper band (ld >= b+1) -> working band (ld_w >= b + 2 TW + 1
//               rows per column: tw sub-diagonals of bulge fill, b + tw super-
//               diagonals; storage paragraph of Sec. IV), zero fill, type convert.
//   bb_stage    one bandwidth-reduction stage of Algorithm 1 as a persistent
//               kernel: workgroups claim sweeps in order and chase their bulges
//               step by step; device progress counters replace the paper's
//               kernel relaunch per cycle (Sec. III-A) as the sweep-to-sweep
//               synchronisation.
//   bb_extract  d_i = A(i,i), e_i = A(i,i+1) -> FP64.
//
// Working band addressing: A(i, q) = W[uo + i + q * S] with S = ld_w - 1, i.e.
// column q of the band is contiguous and holds rows q - uo .. q - uo + ld_w - 1.
//
// Step geometry of sweep r in a stage (b, tw, c) (0-based, derived from Alg. 1):
//   step 0 : k = r,               p = r + c, m = min(r + b, n-1) - p
//   step j : k = r + c + (j-1) b, p = k + b, m = min(tw, n-1-p),  j = 1 .. J-1
// Right task of a step (Alg. 1 first HH line, Alg. 2 lines 3-13): reflector from
// A[k, p..p+m], applied to rows k+1 .. p+m.  Left task (second HH line, Alg. 2
// line 15): reflector from A[p..p+m, p], applied to columns p+1 .. min(p+m+b, n-1).
//
// Scheduling: half-step h = 2j is the right task of step j, h = 2j+1 the left
// one.  Half-step h of sweep r waits until sweep r-1 has completed h + H half-
// steps (or is done), where H depends only on c = b - tw: 2 for c >= 3, 3 for
// c = 2, 4 for c = 1.  Concurrently running tasks then touch disjoint data, so
// the result equals the sequential order of Algorithm 1 up to the rounding of
// each task's own arithmetic.  (The paper's rule, Sec. III-A, is three full
// cycles, i.e. H = 6; splitting a step into its two tasks and making "done"
// transitive is what allows the shorter lag.)
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "bb_device.h"
#include "bb_internal.h"

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
// pack / extract / fill
// ---------------------------------------------------------------------------
template <typename T>
__global__ void bb_pack(const T* __restrict__ band, int64_t ldband, int64_t n, int64_t b_in, int64_t b,
                        T* __restrict__ W, int64_t ldw, int64_t uo, float scale) {
    const int64_t total = n * ldw;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t q = idx / ldw, o = idx - q * ldw;
        const int64_t i = q - uo + o;  // row held at offset o of column q
        T v = T(0);
        if (i >= 0 && i <= q && q - i <= b) {
            v = band[(b_in + i - q) + q * ldband];
            if (scale != 1.0f) v = static_cast<T>(static_cast<float>(v) * scale);
        }
        W[idx] = v;
    }
}

template <typename T>
__global__ void bb_extract(const T* __restrict__ W, int64_t n, int64_t ldw, int64_t uo, double inv_scale,
                           double* __restrict__ d, double* __restrict__ e) {
    const T* A = W + uo;
    const int64_t S = ldw - 1;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        d[i] = static_cast<double>(A[i + i * S]) * inv_scale;
        if (i + 1 < n) e[i] = static_cast<double>(A[i + (i + 1) * S]) * inv_scale;
    }
}

// FP16 storage: per-stage power-of-two scale.  amax receives the bit pattern of
// max |W| (non-negative floats order like their bit patterns); the rescale
// kernel then multiplies every entry by 2^(e_new - e_old), where e_new puts
// max |W| in [2^kF16Top, 2^(kF16Top+1)).  Multiplying by a power of two is exact
// unless a value leaves the FP16 range.  exps[s] is the exponent in force
// before stage s's rescale; exps[s+1] after it.
constexpr int kF16Top = 11;

__global__ void bb_absmax_f16(const _Float16* __restrict__ W, int64_t count, unsigned* __restrict__ amax) {
    float m = 0.f;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        m = fmaxf(m, fabsf(static_cast<float>(W[i])));
    for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(amax, __float_as_uint(m));
}

__device__ __forceinline__ int f16_target_exp(unsigned amax_bits, int e_old) {
    const float m = __uint_as_float(amax_bits);
    if (!(m > 0.f) || !isfinite(m)) return e_old;
    return e_old + (kF16Top - ilogbf(m));
}

__global__ void bb_rescale_f16(_Float16* __restrict__ W, int64_t count, const unsigned* __restrict__ amax,
                               int* __restrict__ exps, int s) {
    const int e_old = exps[s];
    const int e_new = f16_target_exp(*amax, e_old);
    if (blockIdx.x == 0 && threadIdx.x == 0) exps[s + 1] = e_new;
    const int de = e_new - e_old;
    if (de == 0) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        W[i] = static_cast<_Float16>(ldexpf(static_cast<float>(W[i]), de));
}

__global__ void bb_extract_f16(const _Float16* __restrict__ W, int64_t n, int64_t ldw, int64_t uo,
                               const int* __restrict__ exps, int nexp, double* __restrict__ d,
                               double* __restrict__ e) {
    const _Float16* A = W + uo;
    const int64_t S = ldw - 1;
    const int ex = exps[nexp];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        d[i] = ldexp(static_cast<double>(A[i + i * S]), -ex);
        if (i + 1 < n) e[i] = ldexp(static_cast<double>(A[i + (i + 1) * S]), -ex);
    }
}

__global__ void bb_fill_i32(int* __restrict__ p, int64_t count, int value) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

// ---------------------------------------------------------------------------
// Householder application to one row / column segment of m+1 values held in
// registers: a <- a - (tau (a . v)) v.
//   FP64 storage: the dot is summed left to right with separate multiply and add
//   and the update is a - (tau w) v, i.e. the same IEEE operations as a plain
//   sequential implementation (no fused multiply-add; contraction is off).
//   FP32 / FP16 storage: compensated Dot2 (Ogita, Rump, Oishi 2005) with
//   TwoSum and an FMA-based TwoProduct, then a - fma(tau w, v).
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
        float s = 0.f, comp = 0.f;
#pragma unroll
        for (int t = 0; t <= TWM; ++t) {
            const float pr = av[t] * vs[t];
            const float ep = fmaf(av[t], vs[t], -pr);
            float es;
            two_sum(s, pr, s, es);
            comp = comp + (es + ep);
        }
        const float tw = tau * (s + comp);
#pragma unroll
        for (int t = 0; t <= TWM; ++t) av[t] = fmaf(-tw, vs[t], av[t]);
    }
}

// ---------------------------------------------------------------------------
// Window segment movement.  Entry t of a segment lives at column / row offset
// min(t, m) (always inside the window); entries t > m are masked to 0 on load
// and re-store the value of entry m on store, so no per-element branch is needed.
// ---------------------------------------------------------------------------
// `base` points at A(k, p) of the current step; in-window offsets fit in 32 bits.
template <typename T, typename C, int TWM>
__device__ __forceinline__ void load_row(C (&av)[TWM + 1], const T* __restrict__ base, int S, int di, int m) {
    const T* row = base + di;  // A(k + di, p + t) = row[t * S]
#pragma unroll
    for (int t = 0; t <= TWM; ++t) {
        const C v = to_c(row[min(t, m) * S]);
        av[t] = t <= m ? v : C(0);
    }
}

template <typename T, typename C, int TWM>
__device__ __forceinline__ void store_row(const C (&av)[TWM + 1], T* __restrict__ base, int S, int di, int m) {
    T* row = base + di;
#pragma unroll
    for (int t = 0; t <= TWM; ++t) row[min(t, m) * S] = static_cast<T>(av[min(t, m)]);
}

// column q = p + 1 + ci of rows p..p+m; columns p+1..p+m come from the LDS corner
// `base` points at A(p, p); column q = p + 1 + ci starts at base + (1 + ci) * S.
template <typename T, typename C, int TWM>
__device__ __forceinline__ void load_col(C (&av)[TWM + 1], const T* __restrict__ base, int S, const C* corner, int ci,
                                         int m) {
    constexpr int LDC = TWM + 1;
    if (ci < m) {
#pragma unroll
        for (int t = 0; t <= TWM; ++t) {
            const C v = corner[min(t, m) * LDC + ci + 1];
            av[t] = t <= m ? v : C(0);
        }
    } else {
        const T* col = base + (1 + ci) * S;  // A(p + t, q) = col[t]
#pragma unroll
        for (int t = 0; t <= TWM; ++t) {
            const C v = to_c(col[min(t, m)]);
            av[t] = t <= m ? v : C(0);
        }
    }
}

template <typename T, typename C, int TWM>
__device__ __forceinline__ void store_col(const C (&av)[TWM + 1], T* __restrict__ base, int S, int ci, int m) {
    T* col = base + (1 + ci) * S;
#pragma unroll
    for (int t = 0; t <= TWM; ++t) col[min(t, m)] = static_cast<T>(av[min(t, m)]);
}

// ---------------------------------------------------------------------------
// one bandwidth-reduction stage
// ---------------------------------------------------------------------------
template <typename T, int TWM, int NT>
__global__ __launch_bounds__(NT) void bb_stage(StageArgs a) {
    using C = typename Compute<T>::type;
    constexpr int LDC = TWM + 1;  // leading dimension of the LDS corner block
    __shared__ C corner[LDC * LDC];
    __shared__ int s_word[2];

    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    T* __restrict__ A = reinterpret_cast<T*>(a.W) + a.uo;
    const int64_t S = a.S;
    const int S32 = (int)a.S;
    const int n = a.n, b = a.b, tw = a.tw, c = a.c, H = a.H;
    const SyncCtx sc{a.abort_flag, a.err_word, a.spin_limit};

    for (;;) {
        if (tid == 0) {
            int r = atomicAdd(a.claim, 1);
            if (__hip_atomic_load(a.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) r = a.nsweeps;
            s_word[0] = r;
        }
        __syncthreads();
        const int r = s_word[0];
        if (r >= a.nsweeps) return;
        const int* prev = r > 0 ? a.progress + (r - 1) : nullptr;
        int* mine = a.progress + r;
        const int nsteps = 1 + (n - 2 - r - c) / b;

        for (int j = 0; j < nsteps; ++j) {
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

            // ------------------------- right (row) task -------------------------
            // reflector from A[k, p..p+m]; applied to rows k+1..p+m of columns p..p+m.
            // Loads are issued before the reflector is formed so their latency overlaps
            // it; column indices are clamped to p+min(t, m) so every access stays in the
            // window without per-element branches, and entries t > m are masked to 0.
            if (prev && !wait_ge(prev, 2 * j + H, sc, &s_word[1])) return;
            {
                const int rows = p + m - k;
                T* base = A + k + (int64_t)p * S;  // A(k, p)
                const double xl = static_cast<double>(base[min(lane, m) * S32]);
                int ri = tid;
                C av[TWM + 1];
                load_row<T, C, TWM>(av, base, S32, 1 + min(ri, rows - 1), m);
                double vd[TWM + 1], taud, betad;
                house_uniform<TWM>(xl, m, vd, taud, betad);
                C vs[TWM + 1];
#pragma unroll
                for (int t = 0; t <= TWM; ++t) vs[t] = static_cast<C>(vd[t]);
                const C tau = static_cast<C>(taud);
                while (ri < rows) {
                    const int i = k + 1 + ri;
                    if (taud != 0.0) apply_segment<C, TWM>(av, vs, tau, m);
                    if (i >= p) {  // bottom (m+1) x (m+1) corner stays on chip for the left task
#pragma unroll
                        for (int t = 0; t <= TWM; ++t) corner[(i - p) * LDC + t] = av[t];
                    } else {
                        store_row<T, C, TWM>(av, base, S32, 1 + ri, m);
                    }
                    ri += NT;
                    if (ri < rows) load_row<T, C, TWM>(av, base, S32, 1 + ri, m);
                }
                // every wave has read row k: now overwrite it with (beta, 0, ..., 0)
                __syncthreads();
                if (tid <= m) base[tid * S32] = static_cast<T>(tid == 0 ? betad : 0.0);
                publish(mine, 2 * j + 1);
            }

            // ------------------------- left (column) task -------------------------
            // reflector from A[p..p+m, p]; applied to rows p..p+m of columns p+1..L.
            // (the corner was completed before the barrier that ended the right task)
            if (prev && !wait_ge(prev, 2 * j + 1 + H, sc, &s_word[1])) return;
            {
                const int L = min(p + m + b, n - 1);
                const int cols = L - p;  // columns p+1 .. L
                int ci = tid;
                T* base = A + p + (int64_t)p * S;  // A(p, p)
                C av[TWM + 1];
                load_col<T, C, TWM>(av, base, S32, corner, min(ci, cols - 1), m);
                const double xl = static_cast<double>(corner[min(lane, m) * LDC]);
                double vd[TWM + 1], taud, betad;
                house_uniform<TWM>(xl, m, vd, taud, betad);
                C vs[TWM + 1];
#pragma unroll
                for (int t = 0; t <= TWM; ++t) vs[t] = static_cast<C>(vd[t]);
                const C tau = static_cast<C>(taud);
                while (ci < cols) {
                    if (taud != 0.0) apply_segment<C, TWM>(av, vs, tau, m);
                    store_col<T, C, TWM>(av, base, S32, ci, m);
                    ci += NT;
                    if (ci < cols) load_col<T, C, TWM>(av, base, S32, corner, ci, m);
                }
                if (tid <= m) base[tid] = static_cast<T>(tid == 0 ? betad : 0.0);
                publish(mine, 2 * j + 2);
            }
        }
        if (prev && !wait_ge(prev, kDone, sc, &s_word[1])) return;
        if (tid == 0) __hip_atomic_store(mine, kDone, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();  // s_word reuse by the next claim
    }
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
template <typename T>
static hipError_t launch_pack_t(const void* band, int64_t ldband, int64_t n, int64_t b_in, int64_t b, void* W,
                                int64_t ldw, int64_t uo, float scale, hipStream_t st) {
    const int64_t total = n * ldw;
    int grid = (int)std::min<int64_t>((total + 255) / 256, 65536);
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(bb_pack<T>, dim3(grid), dim3(256), 0, st, static_cast<const T*>(band), ldband, n, b_in, b,
                       static_cast<T*>(W), ldw, uo, scale);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_extract_t(const void* W, int64_t n, int64_t ldw, int64_t uo, double inv_scale, double* d,
                                   double* e, hipStream_t st) {
    int grid = (int)std::min<int64_t>((n + 255) / 256, 65536);
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(bb_extract<T>, dim3(grid), dim3(256), 0, st, static_cast<const T*>(W), n, ldw, uo, inv_scale,
                       d, e);
    return hipGetLastError();
}

hipError_t launch_pack(int dtype, const void* band, int64_t ldband, int64_t n, int64_t b_in, int64_t b, void* W,
                       int64_t ldw, int64_t uo, float scale, hipStream_t st) {
    switch (dtype) {
        case 0: return launch_pack_t<double>(band, ldband, n, b_in, b, W, ldw, uo, scale, st);
        case 1: return launch_pack_t<float>(band, ldband, n, b_in, b, W, ldw, uo, scale, st);
        default: return launch_pack_t<_Float16>(band, ldband, n, b_in, b, W, ldw, uo, scale, st);
    }
}

hipError_t launch_extract(int dtype, const void* W, int64_t n, int64_t ldw, int64_t uo, double inv_scale, double* d,
                          double* e, hipStream_t st) {
    switch (dtype) {
        case 0: return launch_extract_t<double>(W, n, ldw, uo, inv_scale, d, e, st);
        case 1: return launch_extract_t<float>(W, n, ldw, uo, inv_scale, d, e, st);
        default: return launch_extract_t<_Float16>(W, n, ldw, uo, inv_scale, d, e, st);
    }
}

hipError_t launch_f16_rescale(void* W, int64_t count, unsigned* amax, int* exps, int s, hipStream_t st) {
    int grid = (int)std::min<int64_t>((count + 255) / 256, 2048);
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(bb_fill_i32, dim3(1), dim3(64), 0, st, reinterpret_cast<int*>(amax), (int64_t)1, 0);
    hipLaunchKernelGGL(bb_absmax_f16, dim3(grid), dim3(256), 0, st, static_cast<const _Float16*>(W), count, amax);
    hipLaunchKernelGGL(bb_rescale_f16, dim3(grid), dim3(256), 0, st, static_cast<_Float16*>(W), count,
                       (const unsigned*)amax, exps, s);
    return hipGetLastError();
}

hipError_t launch_extract_f16(const void* W, int64_t n, int64_t ldw, int64_t uo, const int* exps, int nexp,
                              double* d, double* e, hipStream_t st) {
    int grid = (int)std::min<int64_t>((n + 255) / 256, 65536);
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(bb_extract_f16, dim3(grid), dim3(256), 0, st, static_cast<const _Float16*>(W), n, ldw, uo,
                       exps, nexp, d, e);
    return hipGetLastError();
}

hipError_t launch_fill(int* p, int64_t count, int value, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    int grid = (int)std::min<int64_t>((count + 255) / 256, 4096);
    hipLaunchKernelGGL(bb_fill_i32, dim3(grid), dim3(256), 0, st, p, count, value);
    return hipGetLastError();
}

template <typename T, int TWM, int NT>
static hipError_t launch_stage_t(const StageArgs& a, int grid, hipStream_t st) {
    hipLaunchKernelGGL((bb_stage<T, TWM, NT>), dim3(grid), dim3(NT), 0, st, a);
    return hipGetLastError();
}

template <typename T, int TWM>
static hipError_t launch_stage_nt(const StageArgs& a, int nt, int grid, hipStream_t st) {
    switch (nt) {
        case 64: return launch_stage_t<T, TWM, 64>(a, grid, st);
        case 128: return launch_stage_t<T, TWM, 128>(a, grid, st);
        case 256: return launch_stage_t<T, TWM, 256>(a, grid, st);
        case 512: return launch_stage_t<T, TWM, 512>(a, grid, st);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
static hipError_t launch_stage_tw(const StageArgs& a, int twm, int nt, int grid, hipStream_t st) {
    switch (twm) {
        case 8: return launch_stage_nt<T, 8>(a, nt, grid, st);
        case 16: return launch_stage_nt<T, 16>(a, nt, grid, st);
        case 32: return launch_stage_nt<T, 32>(a, nt, grid, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_stage(int dtype, const StageArgs& a, int twm, int nt, int grid, hipStream_t st) {
    switch (dtype) {
        case 0: return launch_stage_tw<double>(a, twm, nt, grid, st);
        case 1: return launch_stage_tw<float>(a, twm, nt, grid, st);
        default: return launch_stage_tw<_Float16>(a, twm, nt, grid, st);
    }
}

}  // namespace bbk
