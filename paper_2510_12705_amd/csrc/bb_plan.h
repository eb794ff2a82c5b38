// bb_plan.h -- host-only planning: stages of the successive band reduction,
// the half-step dependency lag, the algorithmic-bytes model and the autotune
// cache.
#pragma once

#include <stdint.h>

#include <vector>

#include "bb.h"

namespace bbp {

constexpr int kMaxTW = 64;  // widest compiled tile (FP32 / FP16 storage)
// widest tile of a storage type: 32 for FP64, 64 for FP32 / FP16
int max_tw(int dtype);

struct Stage {
    int b;    // bandwidth entering the stage
    int tw;   // inner tilewidth of the stage, min(TW, b - 1)
    int c;    // bandwidth left, b - tw
    int lag;  // half-step lag between consecutive sweeps
};

struct Plan {
    std::vector<Stage> stages;
};

// Stages of Algorithm 1's outer loop: reduce by TW until the band is bidiagonal.
Plan make_plan(int64_t b, int tw);
// The same stages one at a time, without building a Plan: stage_first(b, tw) is
// the first stage (valid iff b > 1), stage_next(s, tw) the one after s (valid
// iff s.c > 1).
Stage stage_first(int64_t b, int tw);
Stage stage_next(const Stage& s, int tw);
int stage_count(int64_t b, int tw);
// Smallest half-step lag H for which concurrently running tasks of consecutive
// sweeps are disjoint (see bb_kernels.hip): 2 for c >= 3, 3 for c = 2, 4 for c = 1.
int min_lag(int c);

int default_tw(int dtype);
int default_threads(int rows, int dtype);
int default_lanes(int threads_per_lane, int dtype);
int kernel_twm(int tw);

// Read + write bytes of the L-shaped window of every step, summed.
double model_bytes(int64_t n, int64_t b, int elem, int tw);
// The same for the symmetric chase (lower-triangle entries of each step's window).
double sym_model_bytes(int64_t n, int64_t b, int elem, int tw);

// autotuned parameters per (n bucket, b, dtype); 0 fields mean automatic
struct Tuned {
    bb_params_t p;
};
bool autotune_lookup(int64_t n, int64_t b, int dtype, Tuned* out);
void autotune_store(int64_t n, int64_t b, int dtype, const Tuned& t);
void autotune_clear();

}  // namespace bbp
