// Batched Crank-Nicolson steps (include/fsd_batch.h): a native executor
// that runs independent problems on several host threads, each driving
// its own HIP stream, with a longest-processing-time-first assignment.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "../../include/fsd_batch.h"
#include "fsd_host.h"

using namespace fsd;

struct fsd_batch_s {
    std::vector<fsd_problem> P;
    std::vector<size_t> off;
    std::vector<double> iters;       // last step's iterations per problem (cost model)
    size_t ws_bytes = 0;
    std::vector<hipStream_t> streams;
    int lanes = 1;
    int graphs = 0;      // fsd_set_graphs of every problem
    bool bound = false;
};

namespace {

size_t al256(size_t v) { return (v + 255) & ~size_t(255); }

// Relative cost of one CN step of problem i: unknowns x sum of log2 of the
// transform lengths (the FFT work per unknown) x (iterations + 3 for the
// right-hand side and the residual passes).
double cost(const fsd_batch_s& b, int i) {
    const fsd_problem P = b.P[i];
    double lg = 0.0;
    for (int a = 0; a < P->dim; ++a) lg += std::log2((double)std::max(2, P->ax[a].L));
    return (double)P->N * lg * (b.iters[i] + 3.0);
}

// Longest processing time first: problems by decreasing cost, each to the
// lane with the smallest load so far.
std::vector<std::vector<int>> assign(const fsd_batch_s& b, int lanes) {
    const int n = (int)b.P.size();
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::vector<double> c(n);
    for (int i = 0; i < n; ++i) c[i] = cost(b, i);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return c[x] > c[y]; });
    std::vector<std::vector<int>> out(lanes);
    std::vector<double> load(lanes, 0.0);
    for (int i : order) {
        const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        out[l].push_back(i);
        load[l] += c[i];
    }
    return out;
}

fsd_status run_step(fsd_batch b, const double* const* u_prev, const double* const* F,
                    const double* const* guess, double* const* u_next, fsd_stats* stats_out) {
    const int n = (int)b->P.size();
    const auto plan = assign(*b, b->lanes);
    std::vector<fsd_stats> st(n);
    std::vector<fsd_status> status(n, FSD_OK);
    std::vector<std::string> errs(n);
    auto lane_fn = [&](int l) {
        hipStream_t s = b->streams[l];
        for (int i : plan[l]) {
            b->P[i]->stream = s;
            status[i] = fsd_cn_step(b->P[i], u_prev[i], F ? F[i] : nullptr,
                                    guess ? guess[i] : nullptr, u_next[i], &st[i]);
            if (status[i] != FSD_OK) errs[i] = fsd_last_error();
        }
        (void)hipStreamSynchronize(s);
    };
    if (b->lanes == 1) {
        lane_fn(0);
    } else {
        std::vector<std::thread> th;
        th.reserve(b->lanes);
        for (int l = 0; l < b->lanes; ++l) th.emplace_back(lane_fn, l);
        for (auto& t : th) t.join();
    }
    fsd_status first = FSD_OK;
    for (int i = 0; i < n; ++i) {
        b->iters[i] = std::max<double>(1.0, (double)st[i].iters);
        if (stats_out) stats_out[i] = st[i];
        if (status[i] != FSD_OK && first == FSD_OK) {
            first = status[i];
            set_error(first, "problem " + std::to_string(i) + ": " + errs[i]);
        }
    }
    return first;
}

}  // namespace

extern "C" {

fsd_status fsd_batch_create(const fsd_params* params, int count, fsd_batch* out) {
    if (!out) return set_error(FSD_EINVAL, "null output handle");
    *out = nullptr;
    if (!params || count < 1) return set_error(FSD_EINVAL, "need count >= 1 parameter sets");
    fsd_batch b = new fsd_batch_s();
    size_t off = 0;
    for (int i = 0; i < count; ++i) {
        fsd_problem p = nullptr;
        const fsd_status s = fsd_init_problem(&params[i], &p);
        if (s != FSD_OK) {
            const std::string msg = std::string("problem ") + std::to_string(i) + ": " + fsd_last_error();
            for (fsd_problem q : b->P) fsd_destroy(q);
            delete b;
            return set_error(s, msg);
        }
        b->P.push_back(p);
        b->off.push_back(off);
        off = al256(off + fsd_workspace_bytes(p));
        b->iters.push_back(8.0);
    }
    b->ws_bytes = off;
    *out = b;
    return FSD_OK;
}

void fsd_batch_destroy(fsd_batch b) {
    if (!b) return;
    for (fsd_problem p : b->P) fsd_destroy(p);
    delete b;
}

size_t fsd_batch_workspace_bytes(fsd_batch b) { return b ? b->ws_bytes : 0; }

size_t fsd_batch_offset(fsd_batch b, int i) {
    if (!b || i < 0 || i >= (int)b->P.size()) return 0;
    return b->off[i];
}

fsd_status fsd_batch_bind(fsd_batch b, void* d_ws, size_t bytes, void* const* streams, int nstreams) {
    if (!b || !d_ws || !streams || nstreams < 1) return set_error(FSD_EINVAL, "null argument");
    if (((uintptr_t)d_ws & 255) != 0) return set_error(FSD_EINVAL, "workspace must be 256-byte aligned");
    if (bytes < b->ws_bytes) return set_error(FSD_ESMALLWS, "workspace smaller than fsd_batch_workspace_bytes()");
    b->streams.assign(nstreams, nullptr);
    for (int l = 0; l < nstreams; ++l) b->streams[l] = static_cast<hipStream_t>(streams[l]);
    const int n = (int)b->P.size();
    for (int i = 0; i < n; ++i) {
        const fsd_status s = fsd_bind(b->P[i], static_cast<char*>(d_ws) + b->off[i],
                                      fsd_workspace_bytes(b->P[i]), b->streams[i % nstreams]);
        if (s != FSD_OK) return set_error(s, "problem " + std::to_string(i) + ": " + fsd_last_error());
    }
    for (int l = 0; l < nstreams; ++l) {
        const hipError_t e = hipStreamSynchronize(b->streams[l]);
        if (e != hipSuccess) return set_error(FSD_EHIP, hipGetErrorString(e));
    }
    b->lanes = std::min(nstreams, n);
    b->bound = true;
    return FSD_OK;
}

fsd_status fsd_batch_set_lanes(fsd_batch b, int lanes) {
    if (!b) return set_error(FSD_EINVAL, "null batch");
    if (!b->bound) return set_error(FSD_ENOTBOUND, "fsd_batch_bind() has not been called");
    if (lanes < 1 || lanes > (int)b->streams.size()) return set_error(FSD_EINVAL, "lanes outside [1, nstreams]");
    b->lanes = lanes;
    return FSD_OK;
}

int fsd_batch_lanes(fsd_batch b) { return b ? b->lanes : 0; }

fsd_status fsd_batch_set_graphs(fsd_batch b, int on) {
    if (!b) return set_error(FSD_EINVAL, "null batch");
    b->graphs = on != 0;
    for (fsd_problem p : b->P) fsd_set_graphs(p, b->graphs);
    return FSD_OK;
}

int fsd_batch_graphs(fsd_batch b) { return b ? b->graphs : 0; }

fsd_status fsd_batch_cn_step(fsd_batch b, const double* const* d_u_prev, const double* const* d_F,
                             const double* const* d_guess, double* const* d_u_next,
                             fsd_stats* stats) {
    if (!b) return set_error(FSD_EINVAL, "null batch");
    if (!b->bound) return set_error(FSD_ENOTBOUND, "fsd_batch_bind() has not been called");
    if (!d_u_prev || !d_u_next) return set_error(FSD_EINVAL, "null vector array");
    return run_step(b, d_u_prev, d_F, d_guess, d_u_next, stats);
}

int fsd_batch_autotune(fsd_batch b, const double* const* d_u_prev, const double* const* d_F,
                       double* const* d_u_next, double* ms_out) {
    if (!b) return -(int)set_error(FSD_EINVAL, "null batch");
    if (!b->bound) return -(int)set_error(FSD_ENOTBOUND, "fsd_batch_bind() has not been called");
    if (!d_u_prev || !d_u_next) return -(int)set_error(FSD_EINVAL, "null vector array");
    const int maxl = std::min((int)b->streams.size(), (int)b->P.size());
    int best = 1, best_g = 0, k = 0;
    double best_ms = 1e300;
    // tile shapes first: every problem's passes on their fastest engines
    for (fsd_problem p : b->P) {
        const fsd_status s = fsd_autotune(p);
        if (s != FSD_OK) return -(int)s;
    }
    // per launch mode (direct launches, then graphs): one untimed step first
    // (tables and caches warm, iteration estimates set, graphs captured),
    // then one timed step per lane count
    for (int g = 0; g < 2; ++g) {
        fsd_batch_set_graphs(b, g);
        b->lanes = maxl;
        fsd_status s = run_step(b, d_u_prev, d_F, nullptr, d_u_next, nullptr);
        if (s != FSD_OK && s != FSD_ENOTCONV) return -(int)s;
        for (int l = 1; l <= maxl; l *= 2, ++k) {
            b->lanes = l;
            const auto t0 = std::chrono::steady_clock::now();
            s = run_step(b, d_u_prev, d_F, nullptr, d_u_next, nullptr);
            const double ms =
                std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            if (s != FSD_OK && s != FSD_ENOTCONV) return -(int)s;
            if (ms_out) ms_out[k] = ms;
            if (ms < best_ms) {
                best_ms = ms;
                best = l;
                best_g = g;
            }
        }
    }
    for (fsd_problem p : b->P) fsd_reset_history(p);
    fsd_batch_set_graphs(b, best_g);
    b->lanes = best;
    return best;
}

fsd_problem fsd_batch_problem(fsd_batch b, int i) {
    if (!b || i < 0 || i >= (int)b->P.size()) return nullptr;
    return b->P[i];
}

}  // extern "C"
