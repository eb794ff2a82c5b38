// bb_internal.h -- declarations shared by the host API and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bbk {

// Arguments of one bandwidth-reduction stage (see bb_kernels.hip).
struct StageArgs {
    void* W;            // working band base (element type = storage type)
    int64_t S;          // ld_w - 1
    int64_t uo;         // offset of the diagonal inside a band column
    int n, b, tw, c, H; // order, bandwidth entering the stage, tilewidth, bandwidth left, half-step lag
    int nsweeps;        // n - c - 1 (sweeps that exist in this stage)
    int* progress;      // [nsweeps] half-step counters (zeroed before launch); only the
                        // last sweep of each group of consecutive sweeps is written
    int* claim;         // [1] next group of sweeps to hand out (zeroed before launch)
    int* abort_flag;    // [1] watchdog abort word (zeroed before launch)
    int* err_word;      // host-mapped error word
    unsigned spin_limit;
};

hipError_t launch_pack(int dtype, const void* band, int64_t ldband, int64_t n, int64_t b_in, int64_t b, void* W,
                       int64_t ldw, int64_t uo, float scale, hipStream_t st);
hipError_t launch_extract(int dtype, const void* W, int64_t n, int64_t ldw, int64_t uo, double inv_scale, double* d,
                          double* e, hipStream_t st);
hipError_t launch_fill(int* p, int64_t count, int value, hipStream_t st);
// FP16 storage: reset amax, reduce max|W|, rescale W by a power of two (exps[s] -> exps[s+1]).
hipError_t launch_f16_rescale(void* W, int64_t count, unsigned* amax, int* exps, int s, hipStream_t st);
hipError_t launch_extract_f16(const void* W, int64_t n, int64_t ldw, int64_t uo, const int* exps, int nexp,
                              double* d, double* e, hipStream_t st);
// largest workgroup (ntl * lanes) the stage kernel variant for tilewidth bound twm accepts
int stage_max_threads(int twm);
// one stage: `lanes` consecutive sweeps per workgroup, `ntl` threads per lane
hipError_t launch_stage(int dtype, const StageArgs& a, int twm, int ntl, int lanes, int grid, hipStream_t st);

}  // namespace bbk
