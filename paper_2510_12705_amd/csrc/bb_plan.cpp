// bb_plan.cpp -- see bb_plan.h.
#include "bb_plan.h"

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>

namespace bbp {

int min_lag(int c) { return c >= 3 ? 2 : (c == 2 ? 3 : 4); }

Stage stage_first(int64_t b, int tw) {
    const int t = (int)std::min<int64_t>(tw, b - 1);
    const int c = (int)(b - t);
    return Stage{(int)b, t, c, min_lag(c)};
}

Stage stage_next(const Stage& s, int tw) { return stage_first(s.c, tw); }

int stage_count(int64_t b, int tw) {
    int k = 0;
    for (int64_t x = b; x > 1; x -= std::min<int64_t>(tw, x - 1)) ++k;
    return k;
}

Plan make_plan(int64_t b, int tw) {
    Plan p;
    if (b > 1)
        for (Stage s = stage_first(b, tw);; s = stage_next(s, tw)) {
            p.stages.push_back(s);
            if (s.c <= 1) break;
        }
    return p;
}

int default_tw(int dtype) { (void)dtype; return 32; }

// threads per window: the smallest power of two (64..256) with one thread per row
// of the window
int default_threads(int rows, int dtype) {
    (void)dtype;
    int nt = 64;
    while (nt < rows && nt < 256) nt *= 2;
    return nt;
}

// sweeps per workgroup: one.  Sweeps sharing a workgroup share its CU's SIMDs,
// so grouping slows every lane more than it saves in hand-over cost once the
// hand-over stays within an XCD's L2.
int default_lanes(int threads_per_lane, int dtype) {
    (void)threads_per_lane;
    (void)dtype;
    return 1;
}

int kernel_twm(int tw) { return tw <= 8 ? 8 : tw <= 16 ? 16 : tw <= 32 ? 32 : 64; }

int max_tw(int dtype) { return dtype == 0 ? 32 : 64; }

// Window of one step (rows k..p+m of columns p..p+m, and rows p..p+m of columns
// p..L) holds (m+1)(L-k+1) elements; it is read and written once.
double model_bytes(int64_t n, int64_t b, int elem, int tw) {
    double elems = 0.0;
    for (const Stage& s : make_plan(b, tw).stages) {
        const int64_t bs = s.b, t = s.tw, c = s.c;
        for (int64_t r = 0; r + c + 1 <= n - 1; ++r) {
            // step 0
            int64_t k = r, p = r + c, m = std::min(r + bs, n - 1) - p;
            int64_t L = std::min(p + m + bs, n - 1);
            elems += (double)(m + 1) * (double)(L - k + 1);
            // steps j >= 1 with p_j = r + c + j*bs; interior ones (m = t, L = p+t+bs) in closed form
            int64_t last_int = n - 1 - t - bs;  // p <= last_int  <=>  interior
            int64_t j_int = (last_int >= r + c + bs) ? (last_int - r - c) / bs : 0;
            elems += (double)j_int * (double)(t + 1) * (double)(2 * bs + t + 1);
            for (int64_t j = j_int + 1;; ++j) {
                p = r + c + j * bs;
                k = p - bs;
                m = std::min(t, n - 1 - p);
                if (m < 1) break;
                L = std::min(p + m + bs, n - 1);
                elems += (double)(m + 1) * (double)(L - k + 1);
            }
        }
    }
    return 2.0 * elems * (double)elem;
}

// Symmetric chase: per step the lower-triangle entries it reads and writes --
// column k's segment, rows p..p+m of the columns k+1..p-1, the block's lower
// triangle, and rows p+m+1..L of columns p..p+m.
double sym_model_bytes(int64_t n, int64_t b, int elem, int tw) {
    double elems = 0.0;
    for (const Stage& s : make_plan(b, tw).stages) {
        const int64_t bs = s.b, t = s.tw, c = s.c;
        for (int64_t r = 0; r + c + 1 <= n - 1; ++r) {
            for (int64_t j = 0;; ++j) {
                const int64_t p = r + c + j * bs;
                const int64_t k = j == 0 ? r : p - bs;
                const int64_t m = j == 0 ? std::min(r + bs, n - 1) - p : std::min(t, n - 1 - p);
                if (m < 1) break;
                const int64_t L = std::min(p + m + bs, n - 1);
                elems += (double)(m + 1) * (double)(p - k) + (double)(m + 1) * (double)(m + 2) / 2.0 +
                         (double)(L - p - m) * (double)(m + 1);
            }
        }
    }
    return 2.0 * elems * (double)elem;
}

namespace {
std::mutex mu;
std::map<std::tuple<int, int64_t, int>, Tuned> cache;
int bucket(int64_t n) {
    int l = 0;
    while ((int64_t(1) << (l + 1)) <= n) ++l;
    return l;
}
}  // namespace

bool autotune_lookup(int64_t n, int64_t b, int dtype, Tuned* out) {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(std::make_tuple(bucket(n), b, dtype));
    if (it == cache.end()) return false;
    *out = it->second;
    return true;
}

void autotune_store(int64_t n, int64_t b, int dtype, const Tuned& t) {
    std::lock_guard<std::mutex> lk(mu);
    cache[std::make_tuple(bucket(n), b, dtype)] = t;
}

void autotune_clear() {
    std::lock_guard<std::mutex> lk(mu);
    cache.clear();
}

}  // namespace bbp
