// bb_device.h -- device-side building blocks for the gfx950 bulge-chasing kernels.
//
// Lane broadcast and the FP64 Householder generator.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bbk {

constexpr int kWave = 64;
constexpr int kDone = 0x7fffffff;  // progress value of a sweep that, and all sweeps before it, finished

// ---------------------------------------------------------------------------
// lane broadcast (full wave active)
// ---------------------------------------------------------------------------
// x on lanes 0..m, +0 on lanes above m
__device__ __forceinline__ double mask_above(double x, int m) {
    return (int)(threadIdx.x & 63) <= m ? x : 0.0;
}

__device__ __forceinline__ double readlane_f64(double x, int lane) {
    int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
    int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
    return __hiloint2double(hi, lo);
}

// ---------------------------------------------------------------------------
// Householder generator (FP64 for every storage type), LAPACK xLARFG.
//
// Every lane of the wave computes the reflector from the same, wave-uniform
// values, in exactly the operation order of the reference definition:
//   xnorm = xNRM2(x2)   (LAPACK >= 3.10: Blue's algorithm, Anderson's constants;
//                        mid-range entries summed as plain squares left to right)
//   xnorm == 0          -> H = I (tau = 0, beta = alpha)
//   beta  = -sign(alpha) xLAPY2(alpha, xnorm), sign(0) = +1
//   |beta| < safmin     -> rescale x by 1/safmin (<= 20 times), recompute
//   tau   = (beta - alpha) / beta,  v = x * (1 / (alpha - beta)),  v0 = 1
// with no fused multiply-add, so FP64 results are bitwise those of a plain
// IEEE double implementation of the same definition.
// ---------------------------------------------------------------------------
#pragma clang fp contract(off)

__device__ __forceinline__ double nrm2_uniform_step(double ax, bool& notbig, double& asml, double& amed,
                                                    double& abig) {
    constexpr double tsml = 0x1p-511, tbig = 0x1p486, ssml = 0x1p537, sbig = 0x1p-538;
    if (ax > tbig) {
        const double y = ax * sbig;
        abig = abig + y * y;
        notbig = false;
    } else if (ax < tsml) {
        if (notbig) {
            const double y = ax * ssml;
            asml = asml + y * y;
        }
    } else {
        amed = amed + ax * ax;
    }
    return ax;
}

__device__ __forceinline__ double nrm2_finish(bool notbig, double asml, double amed, double abig) {
    constexpr double ssml = 0x1p537, sbig = 0x1p-538;
    (void)notbig;
    double scl, sumsq;
    if (abig > 0.0) {
        if (amed > 0.0 || amed != amed) abig = abig + (amed * sbig) * sbig;
        scl = 1.0 / sbig;
        sumsq = abig;
    } else if (asml > 0.0) {
        if (amed > 0.0 || amed != amed) {
            amed = sqrt(amed);
            asml = sqrt(asml) / ssml;
            const double ymin = asml > amed ? amed : asml, ymax = asml > amed ? asml : amed;
            const double q = ymin / ymax;
            scl = 1.0;
            sumsq = ymax * ymax * (1.0 + q * q);
        } else {
            scl = 1.0 / ssml;
            sumsq = asml;
        }
    } else {
        scl = 1.0;
        sumsq = amed;
    }
    return scl * sqrt(sumsq);
}

// General xNRM2 over entries 1..m: entry t < 64 is lane t of xm, entry 64 (only
// with a 65-entry vector) is the wave-uniform xh; each value is first multiplied
// knt times by 2^970 (the xLARFG rescaling).  Rarely taken: a rolled loop reading
// one lane per iteration keeps it small without a call (a call would spill
// registers).
template <bool kHi>
__device__ __forceinline__ double nrm2_lanes_general(double xm, double xh, int m, int knt) {
    constexpr double rsafmn = 2.220446049250313e-16 / 2.2250738585072014e-308;  // 1 / safmin = 2^970
    bool notbig = true;
    double asml = 0.0, amed = 0.0, abig = 0.0;
#pragma unroll 1
    for (int t = 1; t <= m; ++t) {
        double xt = (kHi && t >= kWave) ? xh : readlane_f64(xm, t);
#pragma unroll 1
        for (int i = 0; i < knt; ++i) xt = xt * rsafmn;
        nrm2_uniform_step(fabs(xt), notbig, asml, amed, abig);
    }
    return nrm2_finish(notbig, asml, amed, abig);
}

__device__ __forceinline__ double lapy2(double a, double b) {
    const double xa = fabs(a), ya = fabs(b);
    const double w = xa > ya ? xa : ya, z = xa < ya ? xa : ya;
    if (z == 0.0) return w;
    const double q = z / w;
    return w * sqrt(1.0 + q * q);
}

// x_lane: lane t (0 <= t <= min(m, 63)) holds x_t; with TWM = 64 the 65th entry
// x_64 comes in the wave-uniform x_hi (read only when m = 64).  On return
// v[0..TWM] holds the reflector (v[0] = 1, v[t] = 0 for t > m), equal on every
// lane of the wave, generated through a per-wave LDS scratch `scr` of
// 2 (TWM + 1) doubles: lane t writes x_t^2 and later x_t / (alpha - beta) (lane 0
// also the entries of x_hi), every lane reads them back (broadcast reads), so no
// lane-by-lane register broadcast is needed.  The squares are summed left to
// right in the same order and operations as the plain definition.  All 64 lanes
// of the wave must be active.
// v_own receives this lane's FP64 entry v_lane (0 above m; lane 0's value is not
// v_0 = 1 and is not meant to be used) and v_hi_own the FP64 v_64 of a 65-entry
// vector; the reflector log of the singular-vector path stores them.
template <int TWM, typename V>
__device__ __forceinline__ void house_lds(double x_lane, double x_hi, int m, double* scr, V (&v)[TWM + 1],
                                          double& tau, double& beta, double& v_own, double& v_hi_own) {
    static_assert(TWM <= kWave, "one lane per entry, and one more held wave-uniform");
    constexpr bool kHi = TWM == kWave;
    constexpr double tsml = 0x1p-511, tbig = 0x1p486;
    const int lane = threadIdx.x & (kWave - 1);
    const double xm = mask_above(x_lane, m);  // lanes above m hold +0
    const double xh = kHi && m >= kWave ? x_hi : 0.0;
    double alpha = readlane_f64(xm, 0);
    const double ax = fabs(xm), axh = fabs(xh);
    // every nonzero |x_t| (1 <= t <= m) in [tsml, tbig]: plain sum of squares
    const bool lane_ok = lane == 0 || ax == 0.0 || (ax >= tsml && ax <= tbig);
    const bool hi_ok = axh == 0.0 || (axh >= tsml && axh <= tbig);
    const bool mid = __ballot(!lane_ok) == 0 && hi_ok;
    if (lane <= TWM) scr[lane] = ax * ax;
    if (kHi && lane == 0) scr[kWave] = axh * axh;
    __builtin_amdgcn_wave_barrier();
    double amed = 0.0;
#pragma unroll
    for (int t = 1; t <= TWM; ++t) amed = amed + scr[t];
    double xn = mid ? sqrt(amed) : nrm2_lanes_general<kHi>(xm, xh, m, 0);
    v[0] = V(1);
    if (xn == 0.0) {
#pragma unroll
        for (int t = 1; t <= TWM; ++t) v[t] = V(0);
        tau = 0.0;
        beta = alpha;
        v_own = 0.0;
        v_hi_own = 0.0;
        return;
    }
    double h = lapy2(alpha, xn);
    double bt = alpha >= 0.0 ? -h : h;
    constexpr double safmin = 2.2250738585072014e-308 / 2.220446049250313e-16;  // DBL_MIN / DBL_EPSILON
    constexpr double rsafmn = 1.0 / safmin;
    int knt = 0;
    if (fabs(bt) < safmin) {
        do {
            ++knt;
            bt = bt * rsafmn;
            alpha = alpha * rsafmn;
        } while (fabs(bt) < safmin && knt < 20);
        xn = nrm2_lanes_general<kHi>(xm, xh, m, knt);
        h = lapy2(alpha, xn);
        bt = alpha >= 0.0 ? -h : h;
    }
    const double scal = 1.0 / (alpha - bt);
    double xs = xm, xhs = xh;  // this lane's x_t (and x_64), rescaled like the reference (exact powers of two)
#pragma unroll 1
    for (int i = 0; i < knt; ++i) {
        xs = xs * rsafmn;
        xhs = xhs * rsafmn;
    }
    v_own = xs * scal;  // x_t == 0 for t > m
    v_hi_own = xhs * scal;
    V* sv = reinterpret_cast<V*>(scr + TWM + 1);
    if (lane <= TWM) sv[lane] = static_cast<V>(v_own);
    if (kHi && lane == 0) sv[kWave] = static_cast<V>(v_hi_own);
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int t = 1; t <= TWM; ++t) v[t] = sv[t];
    __builtin_amdgcn_wave_barrier();  // the scratch is rewritten by the next call
    tau = (bt - alpha) / bt;
    for (int i = 0; i < knt; ++i) bt = bt * safmin;
    beta = bt;
}

}  // namespace bbk
