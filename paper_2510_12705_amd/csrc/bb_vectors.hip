// bb_vectors.hip -- the orthogonal factors of the reduction, B = U^T A V.
//
// The paper keeps only the bidiagonal and names the singular vectors as the
// extension (its introduction's closing paragraph and Sec. VII): the reflectors
// that the bulge chase generates must be kept and applied afterwards.  The stage
// kernels log every reflector (tau and v in FP64, v_0 = 1 implicit) of a call
// that asks for the factors; here U = H_1 H_2 ... (the left reflectors in the
// order the reduction applied them) and V likewise from the right reflectors are
// formed by X <- X H_i starting from X = I.
//
// A row x of X is independent of the other rows, so one thread owns one row
// (for tiles up to 32 wide two threads, in two waves of one workgroup, own it,
// each taking every other step of a stage; see bb_backtransform_2w).
// Within a stage the reflectors are taken step by step in decreasing order and,
// for each step j, sweep by sweep in increasing order: the support p..p+m of
// (r, j), p = r + c + j b, then slides by one column per sweep, so the thread
// keeps the row's W = TWM + 1 entries of the current support, and the next few
// columns, in a ring of registers (the loop over sweeps is unrolled over
// the ring so that every index is a compile-time constant) and, per reflector,
// stores the column that leaves the window and loads the one that many
// reflectors ahead; the reflectors themselves are staged through LDS one pass
// over the ring ahead.  Reflectors of one side whose
// supports share a column are met in the same relative order as in the
// reduction (same step: by sweep; different steps: they can only meet when the
// sweep of the larger step comes first), so every entry of X undergoes the same
// operations in the same order as under the sequential order; the dot product
// and the update are the plain sequential ones (no fused multiply-add), so FP64
// results equal a plain sequential accumulation bit for bit (up to the sign of
// zero; a reflector with tau = 0 is applied as the identity it is).  Entries of
// v above m are logged as 0; window slots past column n - 1 hold a copy of
// column n - 1, meet only those zero entries, and are never stored.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "bb_internal.h"

#pragma clang fp contract(off)

namespace bbk {

template <typename T>
using gptr_v = __attribute__((address_space(1))) T*;

constexpr int kWaveLanes = 64;

__global__ void bb_identity(double* __restrict__ X, int64_t n, int64_t ldx) {
    const int64_t total = n * n;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = idx / n, i = idx - j * n;
        X[i + j * ldx] = i == j ? 1.0 : 0.0;
    }
}

// blockIdx.y = 0: V from the right reflectors, 1: U from the left reflectors.
// One wave per workgroup.  For the current reflector (sweep r, support
// p .. p+W-1, p = p0 + r) the thread holds the row's columns p .. p+R-1,
// R = W + ahead: the column that enters at sweep r is loaded `ahead` reflectors
// before its first use, so its latency hides behind that many dot products.
// Reflectors are processed in blocks of kBlk: within a block the register
// holding a column is fixed (reflector u of the block uses x[u .. u+W-1], and
// the column entering behind it goes to x[u+R]), so every index is a
// compile-time constant; after the block the registers move down by kBlk.  The
// reflectors of a block (kBlk consecutive sweeps of one step: kBlk * wlog
// contiguous log entries) sit in one of two LDS buffers; the next block's are
// loaded (coalesced) at the start of a block and written to the other buffer at
// its end.  Keeping the unrolled body to one block keeps the kernel's code well
// inside the instruction cache.
template <int TWM>
constexpr int ring_ahead() { return TWM >= 64 ? 8 : 16; }
constexpr int kBlk = 8;

template <int TWM>
__global__ __launch_bounds__(64) void bb_backtransform(double* __restrict__ Xv, int64_t ldv, double* __restrict__ Xu,
                                                       int64_t ldu, int n, int b, int c, int nsweeps, int nsteps,
                                                       const double* __restrict__ log, int wlog) {
    constexpr int W = TWM + 1;
    constexpr int R = W + ring_ahead<TWM>();
    constexpr int U = kBlk;
    constexpr int BE = U * W;                             // LDS entries of one block (wlog <= W)
    constexpr int Q = (BE + kWaveLanes - 1) / kWaveLanes;  // block entries per lane
    extern __shared__ double vbuf[];                       // [2][U][W]
    double* __restrict__ X = blockIdx.y == 0 ? Xv : Xu;
    const int64_t ldx = blockIdx.y == 0 ? ldv : ldu;
    if (!X) return;
    const int lane = threadIdx.x;
    const int64_t side_slots = (int64_t)nsteps * nsweeps;
    const double* __restrict__ lg = log + (blockIdx.y == 0 ? 0 : side_slots * wlog);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool row = i < n;  // lanes past the last row compute on zeros and store nothing
    gptr_v<double> xi = (gptr_v<double>)(X + (row ? i : 0));
    // Column loads are never predicated (lanes past the last row read row 0, columns past
    // n - 1 read column n - 1), so they land in their registers without a select and
    // their latency stays hidden until first use.  Such values only ever meet zero
    // reflector entries (entries above m are logged as 0) and are never stored.
    auto ld = [&](int col) -> double { return xi[(int64_t)min(col, n - 1) * ldx]; };
    // the block of sweeps r0 .. r0+U-1: entries [u][t], zero beyond wlog or rcount
    auto fetch = [&](const double* __restrict__ slots, int r0, int rcount, double (&q)[Q]) {
#pragma unroll
        for (int z = 0; z < Q; ++z) {
            const int e = lane + kWaveLanes * z;  // entry of the block: u * W + t
            const int u = e / W, t = e - u * W;
            const int r = r0 + u;
            q[z] = (e < BE && t < wlog && r < rcount) ? slots[(int64_t)r * wlog + t] : 0.0;
        }
    };
    auto stage = [&](int buf, const double (&q)[Q]) {
#pragma unroll
        for (int z = 0; z < Q; ++z) {
            const int e = lane + kWaveLanes * z;
            if (e < BE) vbuf[buf * BE + e] = q[z];
        }
        __builtin_amdgcn_wave_barrier();
    };
    for (int j = nsteps - 1; j >= 0; --j) {
        const int rcount = min(n - 1 - c - j * b, nsweeps);  // sweeps with p = r + c + j b <= n - 2
        if (rcount <= 0) continue;
        const int p0 = c + j * b;
        double x[R + U];  // at the start of the block at sweep rb: x[s] = column p0 + rb + s (s < R)
#pragma unroll
        for (int t = 0; t < R; ++t) x[t] = ld(p0 + t);
        const double* __restrict__ slots = lg + (int64_t)j * nsweeps * wlog;
        double q[Q];
        __builtin_amdgcn_wave_barrier();  // the previous step's last block has read its buffer
        fetch(slots, 0, rcount, q);
        stage(0, q);
        int buf = 0;
        for (int rb = 0;; rb += U) {
            fetch(slots, rb + U, rcount, q);  // the next block's reflectors
            const double* vb = vbuf + buf * BE;
            // Every reflector of the block is applied unconditionally: those past rcount
            // (and tau = 0 ones) have tau = 0 and v = 0 in the staged log, so they leave
            // the row unchanged (up to the sign of a zero), and no branch separates the
            // LDS reads of one reflector from the next.
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const double* sl = vb + u * W;
                const double tau = sl[0];
                double w = 0.0;
                w = w + x[u] * 1.0;
#pragma unroll
                for (int t = 1; t < W; ++t) w = w + x[u + t] * sl[t];
                const double tw = tau * w;
                x[u] = x[u] - tw * 1.0;
#pragma unroll
                for (int t = 1; t < W; ++t) x[u + t] = x[u + t] - tw * sl[t];
                // column p leaves the window for good in this step; column p + R enters
                const int p = p0 + rb + u;
                if (row && p < n) xi[(int64_t)p * ldx] = x[u];
                x[u + R] = ld(p + R);
            }
            if (rb + U >= rcount) {
                // the window's remaining columns p0 + rb + U .. + R - 1 sit in x[U ..]
#pragma unroll
                for (int s = U; s < R + U; ++s) {
                    const int col = p0 + rb + s;
                    if (row && col < n) xi[(int64_t)col * ldx] = x[s];
                }
                break;
            }
            stage(buf ^ 1, q);
            buf ^= 1;
#pragma unroll
            for (int t = 0; t < R; ++t) x[t] = x[t + U];
        }
    }
}

// Two steps at a time on two waves (TWM <= 32): wave 0 of a workgroup runs step
// j, wave 1 step j-1, on the same 64 rows, each with its own window and
// reflector stream exactly as above, in block iterations that end with a
// workgroup barrier (which also makes every store of the iteration visible to
// the other wave).  In iteration it wave 0 applies sweeps it U .. it U + U - 1 and
// wave 1 sweeps (it - lag) U ...  Wave 1's window then lies left of every column
// wave 0 holds (lag U >= U + R - b), i.e. on columns wave 0 stored in earlier
// iterations, and two reflectors of the two steps that share a column (r' >=
// r + b - m > r) are met in the reduction's order; with no lag, b - m >= U puts
// them in different iterations.  Each row sees the same operations in the same
// order as with one wave, so the result is bitwise the same.
template <int TWM>
__global__ __launch_bounds__(128) void bb_backtransform_2w(double* __restrict__ Xv, int64_t ldv,
                                                           double* __restrict__ Xu, int64_t ldu, int n, int b, int c,
                                                           int nsweeps, int nsteps, const double* __restrict__ log,
                                                           int wlog) {
    constexpr int W = TWM + 1;
    constexpr int R = W + ring_ahead<TWM>();
    constexpr int U = kBlk;
    constexpr int BE = U * W;
    constexpr int Q = (BE + kWaveLanes - 1) / kWaveLanes;
    extern __shared__ double vbuf[];  // [wave][2][U][W]
    double* __restrict__ X = blockIdx.y == 0 ? Xv : Xu;
    const int64_t ldx = blockIdx.y == 0 ? ldv : ldu;
    if (!X) return;
    const int wv = threadIdx.x / kWaveLanes;
    const int lane = threadIdx.x - wv * kWaveLanes;
    const int64_t side_slots = (int64_t)nsteps * nsweeps;
    const double* __restrict__ lg = log + (blockIdx.y == 0 ? 0 : side_slots * wlog);
    const int64_t i = (int64_t)blockIdx.x * kWaveLanes + lane;
    const bool row = i < n;
    gptr_v<double> xi = (gptr_v<double>)(X + (row ? i : 0));
    auto ld = [&](int col) -> double { return xi[(int64_t)min(col, n - 1) * ldx]; };
    auto fetch = [&](const double* __restrict__ slots, int r0, int rcount, double (&q)[Q]) {
#pragma unroll
        for (int z = 0; z < Q; ++z) {
            const int e = lane + kWaveLanes * z;
            const int u = e / W, t = e - u * W;
            const int r = r0 + u;
            q[z] = (e < BE && t < wlog && r < rcount) ? slots[(int64_t)r * wlog + t] : 0.0;
        }
    };
    double* const vb = vbuf + wv * 2 * BE;
    auto stage = [&](int buf, const double (&q)[Q]) {
#pragma unroll
        for (int z = 0; z < Q; ++z) {
            const int e = lane + kWaveLanes * z;
            if (e < BE) vb[buf * BE + e] = q[z];
        }
        __builtin_amdgcn_wave_barrier();
    };
    const int lag = max(0, (U + R - b + U - 1) / U);
    for (int j = nsteps - 1; j >= 0; j -= 2) {
        const int rca = min(n - 1 - c - j * b, nsweeps);  // sweeps with p <= n - 2
        const int rcb = j >= 1 ? min(n - 1 - c - (j - 1) * b, nsweeps) : 0;
        if (rca <= 0 && rcb <= 0) continue;
        const int la = rca > 0 && rcb > 0 ? lag : 0;
        const int its = max((max(rca, 0) + U - 1) / U, la + (max(rcb, 0) + U - 1) / U);  // same on both waves
        const int jj = wv == 0 ? j : j - 1;
        const int rc = wv == 0 ? rca : rcb;
        const int sh = wv == 0 ? 0 : la;
        const int p0 = c + jj * b;
        const double* __restrict__ slots = lg + (int64_t)max(jj, 0) * nsweeps * wlog;
        double x[R + U];
        double q[Q];
        int buf = 0;
        for (int it = 0; it < its; ++it) {
            const int rb = (it - sh) * U;
            if (rb >= 0 && rb < rc) {  // wave-uniform
                if (rb == 0) {
#pragma unroll
                    for (int t = 0; t < R; ++t) x[t] = ld(p0 + t);
                    fetch(slots, 0, rc, q);
                    stage(0, q);
                    buf = 0;
                }
                fetch(slots, rb + U, rc, q);
                const double* cur = vb + buf * BE;
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const double* sl = cur + u * W;
                    const double tau = sl[0];
                    double w = 0.0;
                    w = w + x[u] * 1.0;
#pragma unroll
                    for (int t = 1; t < W; ++t) w = w + x[u + t] * sl[t];
                    const double tw = tau * w;
                    x[u] = x[u] - tw * 1.0;
#pragma unroll
                    for (int t = 1; t < W; ++t) x[u + t] = x[u + t] - tw * sl[t];
                    const int p = p0 + rb + u;
                    if (row && p < n) xi[(int64_t)p * ldx] = x[u];
                    x[u + R] = ld(p + R);
                }
                if (rb + U >= rc) {
#pragma unroll
                    for (int s2 = U; s2 < R + U; ++s2) {
                        const int col = p0 + rb + s2;
                        if (row && col < n) xi[(int64_t)col * ldx] = x[s2];
                    }
                } else {
                    stage(buf ^ 1, q);
                    buf ^= 1;
#pragma unroll
                    for (int t = 0; t < R; ++t) x[t] = x[t + U];
                }
            }
            __syncthreads();  // this iteration's stores are visible to the other wave
        }
    }
}

hipError_t launch_identity(double* X, int64_t n, int64_t ldx, hipStream_t st) {
    if (!X || n <= 0) return hipSuccess;
    const int grid = (int)std::min<int64_t>((n * n + 255) / 256, 8192);
    hipLaunchKernelGGL(bb_identity, dim3(grid), dim3(256), 0, st, X, n, ldx);
    return hipGetLastError();
}

template <int TWM>
static void launch_bt(dim3 grid, hipStream_t st, double* Xv, int64_t ldv, double* Xu, int64_t ldu, int n, int b, int c,
                      int nsweeps, int nsteps, const double* log, int wlog) {
    const size_t lds = sizeof(double) * 2 * (size_t)kBlk * (TWM + 1);
    hipLaunchKernelGGL(bb_backtransform<TWM>, grid, dim3(kWaveLanes), lds, st, Xv, ldv, Xu, ldu, n, b, c, nsweeps,
                       nsteps, log, wlog);
}

template <int TWM>
static void launch_2w(dim3 grid, hipStream_t st, double* Xv, int64_t ldv, double* Xu, int64_t ldu, int n, int b,
                      int c, int nsweeps, int nsteps, const double* log, int wlog) {
    const size_t lds = sizeof(double) * 4 * (size_t)kBlk * (TWM + 1);
    hipLaunchKernelGGL(bb_backtransform_2w<TWM>, grid, dim3(2 * kWaveLanes), lds, st, Xv, ldv, Xu, ldu, n, b, c,
                       nsweeps, nsteps, log, wlog);
}

hipError_t launch_backtransform(double* Xv, int64_t ldv, double* Xu, int64_t ldu, int n, int b, int tw, int c,
                                int nsweeps, int nsteps, const double* log, int wlog, hipStream_t st) {
    if ((!Xv && !Xu) || n <= 1 || nsweeps <= 0 || nsteps <= 0) return hipSuccess;
    const dim3 grid((unsigned)((n + kWaveLanes - 1) / kWaveLanes), 2);
    if (tw <= 8) launch_2w<8>(grid, st, Xv, ldv, Xu, ldu, n, b, c, nsweeps, nsteps, log, wlog);
    else if (tw <= 16) launch_2w<16>(grid, st, Xv, ldv, Xu, ldu, n, b, c, nsweeps, nsteps, log, wlog);
    else if (tw <= 32) launch_2w<32>(grid, st, Xv, ldv, Xu, ldu, n, b, c, nsweeps, nsteps, log, wlog);
    else if (tw <= 64) launch_bt<64>(grid, st, Xv, ldv, Xu, ldu, n, b, c, nsweeps, nsteps, log, wlog);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace bbk
