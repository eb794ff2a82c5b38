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
    int* claim;         // [1] next group of sweeps to hand out (zeroed before launch); with
                        // nxcd > 0: [nxcd] per-XCD claim counters
    int* abort_flag;    // [1] watchdog abort word (zeroed before launch)
    int* err_word;      // host-mapped error word
    unsigned spin_limit;
    int nxcd;           // XCDs of the device (0: groups are claimed in one global order; the
                        // host passes 0 when the grid is smaller than the XCD count, since
                        // XCD-aware claims need a workgroup on every XCD)
    int xcd_run;        // consecutive groups placed on one XCD (>= 1; used when nxcd > 0)
    double* vlog;       // reflector log (null: none): [side][step j][sweep r][wlog] doubles,
                        // side 0 = right (row) reflectors, 1 = left (column) reflectors;
                        // a slot holds tau, v_1 .. v_{wlog-1} (zero above m)
    int wlog;           // doubles per slot (TW of the call + 1)
};

// Arguments of one stage of the symmetric band -> tridiagonal reduction (bb_sym.hip).
struct SymStageArgs {
    void* W;            // working band, lower layout: A(i, q) = W[(i - q) + q * ldw]
    int64_t ldw;
    int n, b, tw, c, H; // order, bandwidth entering the stage, tilewidth, bandwidth left, step lag
    int nsweeps;        // n - c - 1
    int* progress;      // [nsweeps] steps completed per sweep (zeroed before launch)
    int* claim;         // [1] next sweep to hand out (zeroed before launch)
    int* abort_flag;    // [1] watchdog abort word (zeroed before launch)
    int* err_word;
    unsigned spin_limit;
};
// threads per workgroup of the symmetric stage kernel for a stage (b, tw): 256 or 512
int sym_stage_threads(int b, int tw);
hipError_t launch_sym_stage(int dtype, const SymStageArgs& a, int twm, int nt, int grid, hipStream_t st);
hipError_t launch_sym_pack(int dtype, const void* band, int64_t ldband, int64_t n, int64_t b, void* W, int64_t ldw,
                           hipStream_t st);
hipError_t launch_sym_extract(int dtype, const void* W, int64_t n, int64_t ldw, double* d, double* e, hipStream_t st);

// ---- ragged batch ----
struct BatchStage {
    int b, tw, c, H;   // stage geometry and half-step lag
    int nsweeps;       // n - c - 1
    int ngroups;       // groups of consecutive sweeps
    int prog_off;      // offset of this stage's group progress words
};
struct BatchMatrix {
    void* W;           // working band (element type = storage type)
    int64_t S;         // ld_w - 1
    int64_t uo;        // diagonal offset in a band column
    int n, b, b_in;    // order, clamped bandwidth, caller's bandwidth (band indexing)
    int nstages;
    int stage_off;     // index of the first BatchStage of this matrix
    int exp_off;       // FP16: index of this matrix's nstages + 1 scale exponents
};
struct BatchTask {
    int matrix, stage, group;
};
struct BatchArgs {
    const BatchMatrix* mats;
    const BatchStage* stages;
    const BatchTask* tasks;
    int ntasks;
    int* progress;     // all group progress words (zeroed before launch)
    int* exps;         // FP16 scale exponents (zeroed before launch)
    int* claim;
    int* abort_flag;
    int* err_word;
    unsigned spin_limit;
};
hipError_t launch_batched(int dtype, const BatchArgs& a, int twm, int ntl, int lanes, int grid, hipStream_t st);
hipError_t launch_pack_batched(int dtype, const BatchMatrix* mats, int count, int64_t max_elems,
                               const void* const* bands, const int64_t* ldbands, hipStream_t st);
hipError_t launch_extract_batched(int dtype, const BatchMatrix* mats, int count, int64_t max_n, const int* exps,
                                  double* const* ds, double* const* es, hipStream_t st);

hipError_t launch_pack(int dtype, const void* band, int64_t ldband, int64_t n, int64_t b_in, int64_t b, void* W,
                       int64_t ldw, int64_t uo, float scale, hipStream_t st);
hipError_t launch_extract(int dtype, const void* W, int64_t n, int64_t ldw, int64_t uo, double inv_scale, double* d,
                          double* e, hipStream_t st);
hipError_t launch_fill(int* p, int64_t count, int value, hipStream_t st);
// count elements of the storage type, uniform in [-1, 1) from a hash of (index, seed)
hipError_t launch_fill_synth(int dtype, void* p, int64_t count, uint64_t seed, hipStream_t st);
// FP16 storage: reset amax, reduce max|W|, rescale W by a power of two (exps[s] -> exps[s+1]).
hipError_t launch_f16_rescale(void* W, int64_t count, unsigned* amax, int* exps, int s, hipStream_t st);
hipError_t launch_extract_f16(const void* W, int64_t n, int64_t ldw, int64_t uo, const int* exps, int nexp,
                              double* d, double* e, hipStream_t st);
// Singular vectors: X = I (n x n, leading dimension ldx), then X <- X H for every
// reflector of one side of one stage, from that stage's log (see StageArgs::vlog).
// Xv (from the right reflectors) or Xu (from the left ones) may be null.
hipError_t launch_identity(double* X, int64_t n, int64_t ldx, hipStream_t st);
hipError_t launch_backtransform(double* Xv, int64_t ldv, double* Xu, int64_t ldu, int n, int b, int tw, int c,
                                int nsweeps, int nsteps, const double* log, int wlog, hipStream_t st);
// sigma of bidiag(d, e), descending, by bisection on the Golub-Kahan tridiagonal
hipError_t launch_bidiag_sigma(const double* d, const double* e, int64_t n, double* sigma, hipStream_t st);
// largest workgroup (ntl * lanes) the stage kernel variant for tilewidth bound twm accepts
int stage_max_threads(int twm);
// dynamic LDS bytes of one stage workgroup (lanes corners + per-wave staging blocks)
size_t stage_lds_bytes(int dtype, int twm, int ntl, int lanes);
// one stage: `lanes` consecutive sweeps per workgroup, `ntl` threads per lane
hipError_t launch_stage(int dtype, const StageArgs& a, int twm, int ntl, int lanes, int grid, hipStream_t st);

}  // namespace bbk
