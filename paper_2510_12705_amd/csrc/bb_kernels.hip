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
// Right task of a step (the first of the two Householder applications of a step
// in Algorithm 1; the row reflector and its update in Algorithm 2): reflector from
// A[k, p..p+m], applied to rows k+1 .. p+m.  Left task (the second application;
// Algorithm 2's column reflector): reflector from A[p..p+m, p], applied to columns
// p+1 .. min(p+m+b, n-1).
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
#include "bb_window.h"

namespace bbk {

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

// Synthetic band for timing (autotuner): entries uniform in [-1, 1) from a hash of
// the index (splitmix64 finaliser); the values only need to be generic.
template <typename T>
__global__ void bb_fill_synth(T* __restrict__ p, int64_t count, uint64_t seed) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
        uint64_t z = (uint64_t)i + seed * 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        const double u = (double)(z >> 11) * 0x1p-53;  // [0, 1)
        p[i] = static_cast<T>(2.0 * u - 1.0);
    }
}

__global__ void bb_fill_i32(int* __restrict__ p, int64_t count, int value) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

// ---------------------------------------------------------------------------
// Window segment movement.  Entry t of a segment lives at column / row offset
// min(t, m) (always inside the window); entries t > m are masked to 0 on load,
// so no per-element branch or dynamically indexed register array is needed.
// ---------------------------------------------------------------------------
// `base` points at A(k, p) of the current step; in-window offsets fit in 32 bits.
template <typename T, typename C, int TWM>
__device__ __forceinline__ void load_row(C (&av)[TWM + 1], Rsrc base, int S, int di, int m) {
    // A(k + di, p + t) = base[di + t * S]
#pragma unroll
    for (int t = 0; t <= TWM; ++t) {
        const C v = to_c(buf_ld<T>(base, di, min(t, m) * S));
        av[t] = t <= m ? v : C(0);
    }
}

// Stores run from t = TWM down to 0: an entry t > m (masked to 0) lands on the
// clamped address of entry m first and is then overwritten by entry m itself
// (stores of one thread to one address keep program order).
template <typename T, typename C, int TWM>
__device__ __forceinline__ void store_row(const C (&av)[TWM + 1], Rsrc base, int S, int di, int m) {
#pragma unroll
    for (int t = TWM; t >= 0; --t) buf_st<T>(base, di, min(t, m) * S, static_cast<T>(av[t]));
}

// ---------------------------------------------------------------------------
// one bandwidth-reduction stage
//
// A workgroup owns a group of G consecutive sweeps r0 .. r0+G-1 ("lanes"; lane
// g uses threads [g*NTL, (g+1)*NTL)).  Its lanes advance in lock-step phases:
// in phase P, lane g executes half-step h = P - H*g of sweep r0+g (if that
// half-step exists).  Lane g then always trails lane g-1 by H half-steps, which
// is exactly the dependency rule, so hand-over inside the group needs only the
// workgroup barrier that ends each phase.  Lane 0 depends on the last sweep of
// the previous group through that sweep's progress word (thread 0 polls it and
// then acquires at agent scope); after every phase, once each wave has waited
// for its agent-scope band stores, thread 0 publishes the progress of the
// group's last sweep.  By default a group is one sweep (G = 1), whose phases
// wait in two parts (see run_group).  Concurrently running half-steps (of this
// and of other groups) touch disjoint data, so results are bitwise those of the
// sequential order.
// ---------------------------------------------------------------------------
struct StepGeom {
    int k, p, m;
};

__device__ __forceinline__ StepGeom step_geom(int n, int b, int tw, int c, int r, int j) {
    StepGeom g;
    if (j == 0) {
        g.k = r;
        g.p = r + c;
        g.m = min(r + b, n - 1) - g.p;
    } else {
        g.k = r + c + (j - 1) * b;
        g.p = g.k + b;
        g.m = min(tw, n - 1 - g.p);
    }
    return g;
}

// Reflector log of the singular-vector path: the first wave of a task writes its
// reflector's tau and v_1..v_TWM (FP64, zero above m) to the task's slot of
// `wlog` entries; lane 0 also writes v_64 of a 65-entry reflector.  v_0 = 1 is
// implicit.  `slot` is null when nothing is logged.
template <int TWM>
__device__ __forceinline__ void log_reflector(gptr<double> slot, int wlog, int ltid, double tau, double v_own,
                                              double v_hi_own) {
    if (ltid >= kWave) return;
    if (ltid == 0) slot[0] = tau;
    else if (ltid < wlog) slot[ltid] = v_own;
    if constexpr (TWM >= kWave) {
        if (ltid == 0 && kWave < wlog) slot[kWave] = v_hi_own;
    }
}

// half-steps of sweep r (2 per step); sweep r exists iff r <= n - c - 2
__device__ __forceinline__ int sweep_halfsteps(int n, int b, int c, int r) { return 2 * (1 + (n - 2 - r - c) / b); }

// Right task of one lane: reflector from A[k, p..p+m], applied to rows k+1..p+m of
// columns p..p+m.  Rows p..p+m (the bottom (m+1)^2 corner) go to the lane's LDS
// corner for the left task; row k itself is rewritten by the caller after the
// phase barrier (every wave of the lane has read it by then).  Returns beta.
// With `split`, the caller has only waited for the weaker condition (see
// run_group): rows up to p-2 (row k among them) are final then, so they are
// loaded and the reflector is generated before wait_b() (a workgroup barrier,
// called by every thread) establishes the full condition for the other rows and
// for every store.  wait_b() returns false if the pipeline was aborted.
// With `rowk_now` (a one-wave lane that writes row k in its own phase) the wave
// rewrites row k itself once its reflector has consumed the row.
template <typename T, int TWM, int NTL, typename WaitB>
__device__ __forceinline__ double right_task(T* __restrict__ A, int64_t S, int S32, StepGeom g,
                                             typename Compute<T>::type* corner, double* scr, int ltid,
                                             bool split, bool rowk_now, gptr<double> vlog, int wlog,
                                             WaitB&& wait_b) {
    using C = typename Compute<T>::type;
    constexpr int LDC = TWM + 1;
    const int k = uni(g.k), p = uni(g.p), m = uni(g.m);  // a wave never spans two sweeps
    const int lane = ltid & (kWave - 1);
    const int rows = p + m - k;  // rows k+1 .. p+m
    const Rsrc base = make_rsrc(wave_uniform(A + k + (int64_t)p * S));  // A(k, p)
    const double xl = static_cast<double>(buf_ld<T>(base, min(lane, m) * S32, 0));
    // the 65th entry A(k, p+64) of a 64-wide tile (wave-uniform; used only when m = 64)
    const double xh = TWM >= kWave ? static_cast<double>(buf_ld<T>(base, min(kWave, m) * S32, 0)) : 0.0;
    int ri = ltid;
    C av[TWM + 1];
    const bool early = !split || ri < p - 2 - k;  // row k+1+ri <= p-2
    if (early) load_row<T, C, TWM>(av, base, S32, 1 + min(ri, rows - 1), m);
    C vs[TWM + 1];
    double taud, betad, v_own, v_hi;
    house_lds<TWM>(xl, xh, m, scr, vs, taud, betad, v_own, v_hi);
    if (vlog) log_reflector<TWM>(vlog, wlog, ltid, taud, v_own, v_hi);
    if (!wait_b()) return betad;
    if (rowk_now && ltid <= m) buf_st<T>(base, ltid * S32, 0, static_cast<T>(ltid == 0 ? betad : 0.0));
    if (!early) load_row<T, C, TWM>(av, base, S32, 1 + min(ri, rows - 1), m);
    const C tau = static_cast<C>(taud);
    while (ri < rows) {
        const int i = k + 1 + ri;
        if (taud != 0.0) apply_segment<C, TWM>(av, vs, tau, m);
        if (i >= p) {
#pragma unroll
            for (int t = 0; t <= TWM; ++t) corner[(i - p) * LDC + t] = av[t];
        } else {
            store_row<T, C, TWM>(av, base, S32, 1 + ri, m);
        }
        ri += NTL;
        if (ri < rows) load_row<T, C, TWM>(av, base, S32, 1 + ri, m);
    }
    return betad;
}

// Left task of one lane: reflector from A[p..p+m, p] (held in the corner), applied
// to rows p..p+m of columns p+1..L; writes column p as (beta, 0, ..., 0).
// With `split` (see right_task), columns up to p+b-2 are final under the weaker
// condition: they are loaded, and the reflector (from the corner) generated,
// before wait_b(); the other columns are loaded after it.
// Thread ci of the lane owns column p+1+ci (ci += NTL): its m+1 rows are
// contiguous in memory, so it loads them directly (one base address, immediate
// offsets; columns p+1..p+m come from the corner block instead).  The loads are in
// flight while the reflector is generated.  The updated columns go through the
// wave's LDS block (column-major, pitch TWM+1) and are written back as contiguous
// runs across the wave, so the stores are coalesced.  A wave exchanges data only
// with itself through its block (no barrier).
template <typename T, int TWM, int NTL, typename WaitB>
__device__ __forceinline__ void left_task(T* __restrict__ A, int64_t S, int S32, StepGeom g, int n, int b,
                                          const typename Compute<T>::type* corner,
                                          typename Compute<T>::type* stage, double* scr, int ltid,
                                          bool split, gptr<double> vlog, int wlog, WaitB&& wait_b) {
    using C = typename Compute<T>::type;
    constexpr int LDC = TWM + 1;
    const int p = uni(g.p), m = uni(g.m);  // a wave never spans two sweeps
    const int lane = ltid & (kWave - 1);
    const int wv = ltid / kWave;
    const int cols = min(p + m + b, n - 1) - p;  // columns p+1 .. L
    const gptr<T> colp = to_global(A + p + (int64_t)p * S);  // A(p, p), column p
    C* blk = stage + wv * (kWave * LDC);
    const double xl = static_cast<double>(corner[min(lane, m) * LDC]);
    const double xh = TWM >= kWave ? static_cast<double>(corner[min(kWave, m) * LDC]) : 0.0;
    C av[TWM + 1];
    // Column ci of this thread: global rows (clamped to the window), or the corner.
    // The wave's block of columns c0 .. c0+63 is addressed from its first column
    // (cbase = A(p, p+1+c0)), so the per-lane offsets stay small.
    auto block_base = [&](int c0) { return make_rsrc(wave_uniform(colp + (int64_t)(1 + c0) * S)); };
    auto load_cols = [&](Rsrc cbase, int c0, int ci) {
        const int cg = min(max(ci, m), cols - 1);  // an in-window column for every lane, >= c0
        const int o = (cg - c0) * S32;
#pragma unroll
        for (int t = 0; t <= TWM; ++t) av[t] = to_c(buf_ld<T>(cbase, o, min(t, m)));
    };
    int ci = wv * kWave + lane;
    const int c_first = wv * kWave;
    Rsrc cbase = block_base(c_first);
    // column p+1+ci <= p+b-2, or outside the window (its values are discarded)
    const bool early = !split || ci <= b - 3 || ci >= cols;
    if (c_first < cols && early) load_cols(cbase, c_first, ci);
    C vs[TWM + 1];
    double taud, betad, v_own, v_hi;
    house_lds<TWM>(xl, xh, m, scr, vs, taud, betad, v_own, v_hi);
    if (vlog) log_reflector<TWM>(vlog, wlog, ltid, taud, v_own, v_hi);
    if (!wait_b()) return;
    if (c_first < cols && !early) load_cols(cbase, c_first, ci);
    const C tau = static_cast<C>(taud);
    for (int c0 = c_first; c0 < cols; c0 += NTL, ci += NTL) {
        if (c0 != c_first) {
            cbase = block_base(c0);
            load_cols(cbase, c0, ci);
        }
        if (ci < m) {
#pragma unroll
            for (int t = 0; t <= TWM; ++t) av[t] = corner[t * LDC + ci + 1];
        }
#pragma unroll
        for (int t = 0; t <= TWM; ++t) av[t] = t <= m ? av[t] : C(0);
        if (taud != 0.0) apply_segment<C, TWM>(av, vs, tau, m);
#pragma unroll
        for (int t = 0; t <= TWM; ++t) blk[lane * LDC + t] = av[t];
        __builtin_amdgcn_wave_barrier();
        // Write back.  Store u covers rows 0..TWM-1 of kWave/TWM whole columns
        // (lane -> column u*CPI + lane/TWM, row lane%TWM): contiguous runs, and a
        // per-lane offset that is fixed plus a wave-uniform stride.  Row TWM of all
        // kWave columns follows in one more store.  Every LDS slot is read before
        // the stores, so they issue back to back.
        {
            constexpr int CPI = kWave / TWM;
            const int sub = lane / TWM, t = lane % TWM;
            const int cmax = cols - c0;
#pragma unroll
            for (int u = 0; u < TWM; ++u) av[u] = blk[(u * CPI + sub) * LDC + t];
            av[TWM] = blk[lane * LDC + TWM];
            const int o = sub * S32 + t;
            // the stride is made opaque here so that the per-store offsets are formed
            // at the stores instead of being kept live in scalar registers across phases
            int step = CPI * S32;
            asm volatile("" : "+s"(step));
            if (m == TWM && cmax >= kWave) {  // whole block: no per-store predicate
#pragma unroll
                for (int u = 0; u < TWM; ++u) buf_st<T>(cbase, o, u * step, static_cast<T>(av[u]));
                buf_st<T>(cbase, lane * S32, TWM, static_cast<T>(av[TWM]));
            } else {
#pragma unroll
                for (int u = 0; u < TWM; ++u)
                    if (t <= m && u * CPI + sub < cmax) buf_st<T>(cbase, o, u * step, static_cast<T>(av[u]));
                if (m == TWM && lane < cmax) buf_st<T>(cbase, lane * S32, TWM, static_cast<T>(av[TWM]));
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
    if (ltid <= m) buf_st<T>(make_rsrc(wave_uniform(colp)), ltid, 0, static_cast<T>(ltid == 0 ? betad : 0.0));
}

// LDS of one lane (bytes): its (TWM+1)^2 corner and one staging block of
// kWave (TWM+1) elements per wave, in the compute type; then per wave a
// reflector scratch of 2 (TWM+1) doubles.
constexpr size_t lds_align(size_t x) { return (x + 15) / 16 * 16; }
template <typename C, int TWM, int NTL>
struct LaneLds {
    static constexpr int LDC = TWM + 1;
    static constexpr size_t corner = 0;
    static constexpr size_t stage = lds_align(sizeof(C) * LDC * LDC);
    static constexpr size_t scratch = stage + lds_align(sizeof(C) * NTL * LDC);
    static constexpr size_t scratch_per_wave = sizeof(double) * 2 * LDC;
    static constexpr size_t bytes = lds_align(scratch + scratch_per_wave * (NTL / kWave));
};

// Largest workgroup a variant is compiled for.  Wider windows need more
// registers: at 256 threads (one wave per SIMD) the TW <= 32 variant may use more
// than 256 registers per lane, so the compiler keeps its overflow in the
// accumulation registers instead of spilling to scratch memory.
template <int TWM>
constexpr int max_threads() { return TWM >= 32 ? 256 : (TWM >= 16 ? 512 : 1024); }

// One group of consecutive sweeps r0 .. r0+nl-1 of one stage.
struct GroupArgs {
    void* A;                 // working band base + uo (element type T)
    int64_t S;               // ld_w - 1
    int n, b, tw, c, H;      // stage geometry and half-step lag
    int nsweeps;             // sweeps of the stage
    int r0;                  // first sweep of the group
    const int* prev;         // progress word of the previous group of this stage (null: none)
    const int* stage_prev;   // progress word of the last group of the previous stage; must be
                             // DONE before phase 0 (null: no wait)
    int* last;               // this group's progress word
    double* vlog;            // reflector log of this stage (null: not logged): right-task slots
                             // [j][r] then left-task slots [j][r], wlog doubles each
    int wlog;
    int* abort_flag;
    int* err_word;
    unsigned spin_limit;
};

// Executed by the whole workgroup (G lanes of NTL threads).  In phase P lane g
// runs half-step P - H*g of sweep r0+g; see bb_stage below.  Returns false if the
// pipeline was aborted.
template <typename T, int TWM, int NTL, bool LOG>
__device__ bool run_group(const GroupArgs& ga, unsigned char* lds, int* s_ok) {
    // threads 0..m of a lane write a row / column segment of m + 1 <= TWM + 1 entries
    static_assert(NTL > TWM, "a 64-wide tile needs at least two waves per lane");
    using C = typename Compute<T>::type;
    constexpr int LDC = TWM + 1;
    const int tid = threadIdx.x;
    const int G = blockDim.x / NTL;
    const int g = tid / NTL;
    const int ltid = tid - g * NTL;
    using Lay = LaneLds<C, TWM, NTL>;
    unsigned char* my = lds + g * Lay::bytes;
    C* corner = reinterpret_cast<C*>(my + Lay::corner);
    C* stage = reinterpret_cast<C*>(my + Lay::stage);
    double* scr = reinterpret_cast<double*>(my + Lay::scratch + Lay::scratch_per_wave * ((tid - g * NTL) / kWave));
    T* __restrict__ A = reinterpret_cast<T*>(ga.A);
    const int64_t S = ga.S;
    const int S32 = (int)ga.S;
    const int n = ga.n, b = ga.b, tw = ga.tw, c = ga.c, H = ga.H;
    const int r0 = ga.r0;
    const int nl = min(G, ga.nsweeps - r0);
    const int64_t side_slots = (int64_t)(sweep_halfsteps(n, b, c, 0) / 2) * ga.nsweeps;  // steps x sweeps
    const int r = r0 + g;
    const bool has_sweep = g < nl;
    const int len = has_sweep ? sweep_halfsteps(n, b, c, r) : 0;
    // lengths never grow with r, so lane 0 finishes last among the lanes of equal
    // length; phases run until every lane finished
    int P_end = 0;
    for (int l = 0; l < nl; ++l) P_end = max(P_end, sweep_halfsteps(n, b, c, r0 + l) + H * l);
    const int len_prev = ga.prev ? sweep_halfsteps(n, b, c, r0 - 1) : 0;
    const int len_last = sweep_halfsteps(n, b, c, r0 + nl - 1);
    int known = 0;      // thread 0: progress value last seen for the previous group
    int published = 0;  // thread 0: progress value last published for this group

    if (tid == 0) {
        int ok = 1;
        if (ga.stage_prev && poll_ge(ga.stage_prev, kDone, ga.abort_flag, ga.err_word, ga.spin_limit) < 0) ok = 0;
        *s_ok = ok;
    }
    // (the first phase's barrier publishes *s_ok)

    // Row k of a right task is rewritten in the lane's next phase (its left task)
    // when no half-step that the lag rule lets run before that phase ends touches
    // those entries.  An exhaustive happens-before check of the rule (every pair of
    // half-steps of a stage that it leaves unordered must be disjoint; sweep r-i is
    // then only known to have completed h + i (H - 1) + 1 half-steps) shows this
    // for c = 2 and c >= 4; for c = 1 and c = 3 a half-step of a sweep three behind
    // can reach row k, so there the row is written after an extra barrier in the
    // same phase.
    const bool defer_rowk = c == 2 || c >= 4;
    // With one sweep per workgroup the wait of a phase is split in two.  Once the
    // previous sweep has completed h + H - 1 half-steps (one less than the rule
    // asks), the rows of a right task up to p-2 and the columns of a left task up
    // to p+b-2 are final: an exhaustive check of the schedule shows every earlier
    // half-step that touches them is complete by then, for every stage shape.
    // They are loaded and the reflector is generated first; the rest of the window
    // is loaded, and everything is stored, only after the full wait.
    // (Measured: with c = 1, where the lag is 4 half-steps, the extra wait and
    // barrier cost more than the early loads save, so that stage keeps one wait.)
    const bool split = G == 1 && ga.prev != nullptr && c >= 2;
    // A lane of one wave that writes row k in the same phase needs no barrier for
    // it: no other wave reads the row, and the wave has consumed it by then.
    const bool rowk_now = !defer_rowk && NTL == kWave;
    double beta_row = 0.0;
    for (int P = 0; P < P_end; ++P) {
        // ---- dependency on the previous group (thread 0 polls, then acquires) ----
        int need_b = 0;  // thread 0: the full condition of this phase
        if (tid == 0 && *s_ok && ga.prev) {
            int need = 0;
            for (int l = 0; l < nl; ++l) {
                const int h = P - H * l;
                const int ll = sweep_halfsteps(n, b, c, r0 + l);
                if (h < 0 || h >= ll) continue;
                const int pred_len = l == 0 ? len_prev : sweep_halfsteps(n, b, c, r0 + l - 1);
                if (h + H > pred_len) need = kDone;        // predecessor must be DONE
                else if (l == 0) need = max(need, h + H);  // lanes > 0 are covered by lock-step
            }
            need_b = need;
            if (split && need > 0) need = P + H - 1 > len_prev ? kDone : P + H - 1;
            if (need > known) {
                const int v = poll_ge(ga.prev, need, ga.abort_flag, ga.err_word, ga.spin_limit);
                if (v < 0) *s_ok = 0;
                else known = v;
            }
        }
        __syncthreads();
        if (!*s_ok) return false;
        bool waited = false;
        auto wait_b = [&]() -> bool {  // every thread of the workgroup
            waited = true;
            if (!split) return true;
            if (tid == 0 && *s_ok && need_b > known) {
                const int v = poll_ge(ga.prev, need_b, ga.abort_flag, ga.err_word, ga.spin_limit);
                if (v < 0) *s_ok = 0;
                else known = v;
            }
            __syncthreads();
            return *s_ok != 0;
        };

        // ---- this phase's half-step of every lane ----
        const int h = P - H * g;
        const bool active = has_sweep && h >= 0 && h < len;
        StepGeom sg{0, 0, 0};
        if (active) {
            sg = step_geom(n, b, tw, c, r, h >> 1);
            gptr<double> slot = nullptr;
            if constexpr (LOG)
                slot = to_global(ga.vlog) +
                       (((h & 1) * side_slots + (int64_t)(h >> 1) * ga.nsweeps + r) * (int64_t)ga.wlog);
            if ((h & 1) == 0) {
                beta_row = right_task<T, TWM, NTL>(A, S, S32, sg, corner, scr, ltid, split, rowk_now, slot, ga.wlog,
                                                   wait_b);
            } else {
                // row k of this step's right task (read by every wave of the lane in
                // the previous phase) becomes (beta, 0, ..., 0), after the full wait
                auto wait_b_rowk = [&]() -> bool {
                    if (!wait_b()) return false;
                    if (defer_rowk && ltid <= sg.m)
                        st_agent(to_global(A) + (sg.k + (int64_t)(sg.p + ltid) * S),
                                 static_cast<T>(ltid == 0 ? beta_row : 0.0));
                    return true;
                };
                left_task<T, TWM, NTL>(A, S, S32, sg, n, b, corner, stage, scr, ltid, split, slot, ga.wlog,
                                       wait_b_rowk);
            }
        }
        if (!waited) wait_b();  // keeps the barrier count equal when no task ran
        if (!*s_ok) return false;
        if (!defer_rowk && !rowk_now) {
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();  // every wave of every lane has read its row k
            if (active && (h & 1) == 0 && ltid <= sg.m)
                st_agent(to_global(A) + (sg.k + (int64_t)(sg.p + ltid) * S), static_cast<T>(ltid == 0 ? beta_row : 0.0));
        }
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();  // phase complete: its stores are visible inside the workgroup

        // ---- publish the progress of this group's last sweep ----
        if (tid == 0) {
            const int done_last = min(max(P + 1 - H * (nl - 1), 0), len_last);
            if (done_last > published) {
                // every wave waited for its (agent-scope) stores before the barrier
                __hip_atomic_store(ga.last, done_last, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                published = done_last;
            }
        }
    }
    // ---- all sweeps of the group finished: DONE once the previous group is DONE ----
    if (tid == 0) {
        int ok = *s_ok;
        if (ok && ga.prev && known < kDone && poll_ge(ga.prev, kDone, ga.abort_flag, ga.err_word, ga.spin_limit) < 0)
            ok = 0;
        if (ok) {
            __hip_atomic_store(ga.last, kDone, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        *s_ok = ok;
    }
    __syncthreads();
    return *s_ok != 0;
}

// ---------------------------------------------------------------------------
// One bandwidth-reduction stage of one band.  Workgroups claim groups of G
// consecutive sweeps in order (group q depends only on group q-1, claimed
// earlier by a running workgroup, so the claim order cannot deadlock).
// progress[q] is group q's word: half-steps completed by its last sweep, then
// kDone once it and every earlier group finished.
// ---------------------------------------------------------------------------
template <typename T, int TWM, int NTL, bool LOG>
__global__ __launch_bounds__(max_threads<TWM>()) void bb_stage(StageArgs a) {
    using C = typename Compute<T>::type;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    unsigned char* lds = smem_raw;  // G lane blocks
    __shared__ int s_group;
    __shared__ int s_ok;
    const int G = blockDim.x / NTL;
    const int ngroups = (a.nsweeps + G - 1) / G;
    // XCD-aware order: runs of xcd_run consecutive groups are assigned to the XCDs
    // round-robin and each XCD claims its own groups in increasing order, so the
    // hand-over inside a run stays in one L2.  The smallest unfinished group is
    // always claimable (its XCD claimed every earlier group of its sequence), so
    // the claim order cannot deadlock while every XCD holds a workgroup.
    const int Q = a.xcd_run;
    int xcd = 0;
    if (a.nxcd > 0) {
        unsigned id;
        asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(id));
        xcd = (int)((id & 0xfu) % (unsigned)a.nxcd);
    }
    for (;;) {
        if (threadIdx.x == 0) {
            int q;
            if (a.nxcd > 0) {
                const int k = atomicAdd(a.claim + xcd, 1);
                const int64_t qq = ((int64_t)(k / Q) * a.nxcd + xcd) * Q + (k % Q);
                q = qq < ngroups ? (int)qq : ngroups;
            } else {
                q = atomicAdd(a.claim, 1);
            }
            if (__hip_atomic_load(a.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) q = ngroups;
            s_group = q;
        }
        __syncthreads();
        const int q = s_group;
        if (q >= ngroups) return;
        GroupArgs ga;
        ga.A = reinterpret_cast<T*>(a.W) + a.uo;
        ga.S = a.S;
        ga.n = a.n;
        ga.b = a.b;
        ga.tw = a.tw;
        ga.c = a.c;
        ga.H = a.H;
        ga.nsweeps = a.nsweeps;
        ga.r0 = q * G;
        ga.prev = q > 0 ? a.progress + (q - 1) : nullptr;
        ga.stage_prev = nullptr;
        ga.last = a.progress + q;
        ga.vlog = a.vlog;
        ga.wlog = a.wlog;
        ga.abort_flag = a.abort_flag;
        ga.err_word = a.err_word;
        ga.spin_limit = a.spin_limit;
        if (!run_group<T, TWM, NTL, LOG>(ga, lds, &s_ok)) return;
    }
}

// ---------------------------------------------------------------------------
// Ragged batch: one persistent launch over every (matrix, stage, group) task of
// many independent bands.  Tasks are ordered by (stage, group, matrix), so a
// task's dependencies -- the previous group of its stage, and for group 0 the
// last group of the previous stage -- always precede it in the claim order.
// FP16 storage: the workgroup that runs group 0 of a stage first rescales that
// matrix's working band by a power of two (the stage's scale).
// ---------------------------------------------------------------------------
template <typename T, int TWM, int NTL>
__global__ __launch_bounds__(max_threads<TWM>()) void bb_stage_batched(BatchArgs a) {
    using C = typename Compute<T>::type;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    unsigned char* lds = smem_raw;
    __shared__ int s_task;
    __shared__ int s_ok;
    __shared__ float s_red[32];
    for (;;) {
        if (threadIdx.x == 0) {
            int t = atomicAdd(a.claim, 1);
            if (__hip_atomic_load(a.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) t = a.ntasks;
            s_task = t;
        }
        __syncthreads();
        const int t = s_task;
        if (t >= a.ntasks) return;
        const BatchTask tk = a.tasks[t];
        const BatchMatrix& M = a.mats[tk.matrix];
        const BatchStage& St = a.stages[M.stage_off + tk.stage];
        GroupArgs ga;
        ga.A = reinterpret_cast<T*>(M.W) + M.uo;
        ga.S = M.S;
        ga.n = M.n;
        ga.b = St.b;
        ga.tw = St.tw;
        ga.c = St.c;
        ga.H = St.H;
        ga.nsweeps = St.nsweeps;
        ga.r0 = tk.group * (int)(blockDim.x / NTL);
        ga.prev = tk.group > 0 ? a.progress + St.prog_off + tk.group - 1 : nullptr;
        ga.stage_prev = nullptr;
        if (tk.group == 0 && tk.stage > 0) {
            const BatchStage& Sp = a.stages[M.stage_off + tk.stage - 1];
            ga.stage_prev = a.progress + Sp.prog_off + Sp.ngroups - 1;
        }
        ga.last = a.progress + St.prog_off + tk.group;
        ga.vlog = nullptr;
        ga.wlog = 0;
        ga.abort_flag = a.abort_flag;
        ga.err_word = a.err_word;
        ga.spin_limit = a.spin_limit;
        if constexpr (std::is_same<T, _Float16>::value) {
            if (tk.group == 0) {
                // the previous stage must be complete before the band is rescaled
                if (threadIdx.x == 0) {
                    int ok = 1;
                    if (ga.stage_prev && poll_ge(ga.stage_prev, kDone, a.abort_flag, a.err_word, a.spin_limit) < 0) ok = 0;
                    s_ok = ok;
                }
                __syncthreads();
                if (!s_ok) return;
                ga.stage_prev = nullptr;
                gptr<_Float16> W = to_global(reinterpret_cast<_Float16*>(M.W));
                const int64_t count = (int64_t)M.n * (M.S + 1);
                float mx = 0.f;
                for (int64_t i = threadIdx.x; i < count; i += blockDim.x) mx = fmaxf(mx, fabsf(static_cast<float>(W[i])));
                for (int o = 32; o >= 1; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
                if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = mx;
                __syncthreads();
                if (threadIdx.x == 0) {
                    float m2 = 0.f;
                    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) m2 = fmaxf(m2, s_red[w]);
                    const int e_old = to_global(a.exps)[M.exp_off + tk.stage];
                    int e_new = e_old;
                    if (m2 > 0.f && isfinite(m2)) e_new = e_old + (kF16Top - ilogbf(m2));
                    st_agent(to_global(a.exps) + (M.exp_off + tk.stage + 1), e_new);
                    s_red[0] = __int_as_float(e_new - e_old);
                }
                __syncthreads();
                const int de = __float_as_int(s_red[0]);
                if (de != 0)
                    for (int64_t i = threadIdx.x; i < count; i += blockDim.x)
                        st_agent(W + i, static_cast<_Float16>(ldexpf(static_cast<float>(W[i]), de)));
                __builtin_amdgcn_s_waitcnt(0);
                __syncthreads();
            }
        }
        if (!run_group<T, TWM, NTL, false>(ga, lds, &s_ok)) return;
    }
}

// pack / extract for a batch: the y dimension of the grid strides over the matrices
template <typename T>
__global__ void bb_pack_batched(const BatchMatrix* __restrict__ mats, int count, const void* const* __restrict__ bands,
                                const int64_t* __restrict__ ldbands) {
    for (int mi = blockIdx.y; mi < count; mi += gridDim.y) {
        const BatchMatrix& M = mats[mi];
        const T* band = static_cast<const T*>(bands[mi]);
        const int64_t ldband = ldbands[mi];
        T* W = static_cast<T*>(M.W);
        const int64_t ldw = M.S + 1, total = (int64_t)M.n * ldw;
        for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
             idx += (int64_t)gridDim.x * blockDim.x) {
            const int64_t q = idx / ldw, o = idx - q * ldw;
            const int64_t i = q - M.uo + o;
            T v = T(0);
            if (i >= 0 && i <= q && q - i <= M.b) v = band[(M.b_in + i - q) + q * ldband];
            W[idx] = v;
        }
    }
}

template <typename T>
__global__ void bb_extract_batched(const BatchMatrix* __restrict__ mats, int count, const int* __restrict__ exps,
                                   double* const* __restrict__ ds, double* const* __restrict__ es) {
    for (int mi = blockIdx.y; mi < count; mi += gridDim.y) {
        const BatchMatrix& M = mats[mi];
        const T* A = static_cast<const T*>(M.W) + M.uo;
        const int64_t S = M.S;
        const int ex = exps ? exps[M.exp_off + M.nstages] : 0;
        double* d = ds[mi];
        double* e = es[mi];
        for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < M.n;
             i += (int64_t)gridDim.x * blockDim.x) {
            d[i] = ldexp(static_cast<double>(A[i + i * S]), -ex);
            if (i + 1 < M.n) e[i] = ldexp(static_cast<double>(A[i + (i + 1) * S]), -ex);
        }
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

hipError_t launch_fill_synth(int dtype, void* p, int64_t count, uint64_t seed, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    const int grid = (int)std::min<int64_t>((count + 255) / 256, 4096);
    switch (dtype) {
        case 0: hipLaunchKernelGGL(bb_fill_synth<double>, dim3(grid), dim3(256), 0, st, static_cast<double*>(p), count, seed); break;
        case 1: hipLaunchKernelGGL(bb_fill_synth<float>, dim3(grid), dim3(256), 0, st, static_cast<float*>(p), count, seed); break;
        default: hipLaunchKernelGGL(bb_fill_synth<_Float16>, dim3(grid), dim3(256), 0, st, static_cast<_Float16*>(p), count, seed); break;
    }
    return hipGetLastError();
}

hipError_t launch_fill(int* p, int64_t count, int value, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    int grid = (int)std::min<int64_t>((count + 255) / 256, 4096);
    hipLaunchKernelGGL(bb_fill_i32, dim3(grid), dim3(256), 0, st, p, count, value);
    return hipGetLastError();
}

template <typename T, int TWM, int NTL>
static hipError_t launch_stage_t(const StageArgs& a, int lanes, int grid, hipStream_t st) {
    using C = typename Compute<T>::type;
    const size_t smem = (size_t)lanes * LaneLds<C, TWM, NTL>::bytes;
    if (a.vlog)
        hipLaunchKernelGGL((bb_stage<T, TWM, NTL, true>), dim3(grid), dim3(NTL * lanes), smem, st, a);
    else
        hipLaunchKernelGGL((bb_stage<T, TWM, NTL, false>), dim3(grid), dim3(NTL * lanes), smem, st, a);
    return hipGetLastError();
}

template <typename T, int TWM>
static hipError_t launch_stage_nt(const StageArgs& a, int ntl, int lanes, int grid, hipStream_t st) {
    switch (ntl) {
        case 64:
            if constexpr (TWM < kWave) return launch_stage_t<T, TWM, 64>(a, lanes, grid, st);
            return hipErrorInvalidValue;
        case 128: return launch_stage_t<T, TWM, 128>(a, lanes, grid, st);
        case 256: return launch_stage_t<T, TWM, 256>(a, lanes, grid, st);
        default: return hipErrorInvalidValue;
    }
}

// Tile widths 33..64 exist for the reduced-precision storage types only (their
// 65-entry rows fit the registers; FP64 would not).
template <typename T>
static hipError_t launch_stage_tw(const StageArgs& a, int twm, int ntl, int lanes, int grid, hipStream_t st) {
    switch (twm) {
        case 8: return launch_stage_nt<T, 8>(a, ntl, lanes, grid, st);
        case 16: return launch_stage_nt<T, 16>(a, ntl, lanes, grid, st);
        case 32: return launch_stage_nt<T, 32>(a, ntl, lanes, grid, st);
        case 64:
            if constexpr (!std::is_same<T, double>::value) return launch_stage_nt<T, 64>(a, ntl, lanes, grid, st);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

template <typename T, int TWM, int NTL>
static hipError_t launch_batched_t(const BatchArgs& a, int lanes, int grid, hipStream_t st) {
    using C = typename Compute<T>::type;
    const size_t smem = (size_t)lanes * LaneLds<C, TWM, NTL>::bytes;
    hipLaunchKernelGGL((bb_stage_batched<T, TWM, NTL>), dim3(grid), dim3(NTL * lanes), smem, st, a);
    return hipGetLastError();
}

template <typename T, int TWM>
static hipError_t launch_batched_nt(const BatchArgs& a, int ntl, int lanes, int grid, hipStream_t st) {
    switch (ntl) {
        case 64:
            if constexpr (TWM < kWave) return launch_batched_t<T, TWM, 64>(a, lanes, grid, st);
            return hipErrorInvalidValue;
        case 128: return launch_batched_t<T, TWM, 128>(a, lanes, grid, st);
        case 256: return launch_batched_t<T, TWM, 256>(a, lanes, grid, st);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
static hipError_t launch_batched_tw(const BatchArgs& a, int twm, int ntl, int lanes, int grid, hipStream_t st) {
    switch (twm) {
        case 8: return launch_batched_nt<T, 8>(a, ntl, lanes, grid, st);
        case 16: return launch_batched_nt<T, 16>(a, ntl, lanes, grid, st);
        case 32: return launch_batched_nt<T, 32>(a, ntl, lanes, grid, st);
        case 64:
            if constexpr (!std::is_same<T, double>::value) return launch_batched_nt<T, 64>(a, ntl, lanes, grid, st);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_batched(int dtype, const BatchArgs& a, int twm, int ntl, int lanes, int grid, hipStream_t st) {
    if (lanes < 1 || ntl * lanes > stage_max_threads(twm)) return hipErrorInvalidValue;
    switch (dtype) {
        case 0: return launch_batched_tw<double>(a, twm, ntl, lanes, grid, st);
        case 1: return launch_batched_tw<float>(a, twm, ntl, lanes, grid, st);
        default: return launch_batched_tw<_Float16>(a, twm, ntl, lanes, grid, st);
    }
}

template <typename T>
static hipError_t launch_pack_batched_t(const BatchMatrix* mats, int count, int64_t max_elems, const void* const* bands,
                                        const int64_t* ldbands, hipStream_t st) {
    const int gx = (int)std::max<int64_t>(1, std::min<int64_t>((max_elems + 255) / 256, 1024));
    const int gy = std::min(count, 65535);
    hipLaunchKernelGGL(bb_pack_batched<T>, dim3(gx, gy), dim3(256), 0, st, mats, count, bands, ldbands);
    return hipGetLastError();
}

hipError_t launch_pack_batched(int dtype, const BatchMatrix* mats, int count, int64_t max_elems,
                               const void* const* bands, const int64_t* ldbands, hipStream_t st) {
    switch (dtype) {
        case 0: return launch_pack_batched_t<double>(mats, count, max_elems, bands, ldbands, st);
        case 1: return launch_pack_batched_t<float>(mats, count, max_elems, bands, ldbands, st);
        default: return launch_pack_batched_t<_Float16>(mats, count, max_elems, bands, ldbands, st);
    }
}

template <typename T>
static hipError_t launch_extract_batched_t(const BatchMatrix* mats, int count, int64_t max_n, const int* exps,
                                           double* const* ds, double* const* es, hipStream_t st) {
    const int gx = (int)std::max<int64_t>(1, std::min<int64_t>((max_n + 255) / 256, 1024));
    const int gy = std::min(count, 65535);
    hipLaunchKernelGGL(bb_extract_batched<T>, dim3(gx, gy), dim3(256), 0, st, mats, count, exps, ds, es);
    return hipGetLastError();
}

hipError_t launch_extract_batched(int dtype, const BatchMatrix* mats, int count, int64_t max_n, const int* exps,
                                  double* const* ds, double* const* es, hipStream_t st) {
    switch (dtype) {
        case 0: return launch_extract_batched_t<double>(mats, count, max_n, exps, ds, es, st);
        case 1: return launch_extract_batched_t<float>(mats, count, max_n, exps, ds, es, st);
        default: return launch_extract_batched_t<_Float16>(mats, count, max_n, exps, ds, es, st);
    }
}

int stage_max_threads(int twm) {
    return twm >= 64 ? max_threads<64>() : twm >= 32 ? max_threads<32>() : twm >= 16 ? max_threads<16>() : max_threads<8>();
}

size_t stage_lds_bytes(int dtype, int twm, int ntl, int lanes) {
    // same layout as LaneLds<C, TWM, NTL>
    const size_t c = dtype == 0 ? sizeof(double) : sizeof(float);
    const size_t ldc = (size_t)twm + 1;
    const size_t stage = lds_align(c * ldc * ldc);
    const size_t scratch = stage + lds_align(c * (size_t)ntl * ldc);
    return (size_t)lanes * lds_align(scratch + sizeof(double) * 2 * ldc * (size_t)(ntl / kWave));
}

hipError_t launch_stage(int dtype, const StageArgs& a, int twm, int ntl, int lanes, int grid, hipStream_t st) {
    if (lanes < 1 || ntl * lanes > stage_max_threads(twm)) return hipErrorInvalidValue;
    switch (dtype) {
        case 0: return launch_stage_tw<double>(a, twm, ntl, lanes, grid, st);
        case 1: return launch_stage_tw<float>(a, twm, ntl, lanes, grid, st);
        default: return launch_stage_tw<_Float16>(a, twm, ntl, lanes, grid, st);
    }
}

}  // namespace bbk
