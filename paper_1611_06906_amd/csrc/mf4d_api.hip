// C ABI of libmf4d: validation, FED schedule, workspace layout and the
// orchestration of the scale sweep, tensor and FED kernels on one stream.
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "mf4d_internal.h"

using namespace mf4d;

namespace {

constexpr double kTauLimit = 1.0 / 17.0;   // Eq. (20) at unit pixel spacing
constexpr int kSubstepsPerLaunch = 4;

int radius_of(double sigma)
{
    int r = (int)std::ceil(3.0 * sigma);
    return r < 1 ? 1 : r;
}

// Sampled Gaussian of radius r = max(1, ceil(3 sigma)) normalised to unit sum
// (computed in double), and its central first and second differences, laid
// out as full correlation tables: entry t is the tap at offset i = t - R with
// R = r + 1, i.e. G(i), (G(i-1) - G(i+1)) / 2 and G(i-1) - 2 G(i) + G(i+1),
// zero-padded to a multiple of the register window.
void make_taps(double sigma, WinTaps *t)
{
    const int r = radius_of(sigma);
    const int R = r + 1;
    std::vector<double> g(2 * R + 3, 0.0);   // g[i + R + 1] = G(i), zero beyond r
    double sum = 0.0;
    for (int j = -r; j <= r; ++j) sum += std::exp(-(double)j * j / (2.0 * sigma * sigma));
    for (int j = -r; j <= r; ++j) g[j + R + 1] = std::exp(-(double)j * j / (2.0 * sigma * sigma)) / sum;
    auto G = [&](int i) { return (i < -R - 1 || i > R + 1) ? 0.0 : g[i + R + 1]; };
    std::memset(t, 0, sizeof(*t));
    t->R = R;
    t->ntaps = ((2 * R + 1 + kWin - 1) / kWin) * kWin;
    float gs = 0.f;
    for (int k = 0; k <= 2 * R; ++k) {
        const int i = k - R;
        t->g[k] = (float)G(i);
        t->d1[k] = (float)(0.5 * (G(i - 1) - G(i + 1)));
        t->d2[k] = (float)(G(i - 1) - 2.0 * G(i) + G(i + 1));
        gs += t->g[k];
    }
    t->gsum = gs;
}

void make_rho_taps(double rho, RhoTaps *t)
{
    std::memset(t, 0, sizeof(*t));
    if (!(rho > 0.0)) {
        t->r = 0;
        t->g[0] = 1.f;
        return;
    }
    const int r = radius_of(rho);
    double sum = 0.0;
    for (int j = -r; j <= r; ++j) sum += std::exp(-(double)j * j / (2.0 * rho * rho));
    t->r = r;
    for (int j = 0; j <= r; ++j) t->g[j] = (float)(std::exp(-(double)j * j / (2.0 * rho * rho)) / sum);
}

bool valid_tau_max(double tau_max) { return tau_max > 0.0 && tau_max <= kTauLimit; }

int validate(int H, int W, const mf4d_params *p)
{
    if (!p || H < 3 || W < 3 || (long long)H * (long long)W >= (1LL << 31)) return MF4D_EINVAL;
    if (p->nscales < 1 || p->nscales > MF4D_MAX_SCALES || !p->sigmas) return MF4D_EINVAL;
    for (int s = 0; s < p->nscales; ++s) {
        const float v = p->sigmas[s];
        if (!(v > 0.f) || !std::isfinite(v) || radius_of(v) > MF4D_MAX_RADIUS) return MF4D_EINVAL;
        if (s > 0 && !(v > p->sigmas[s - 1])) return MF4D_EINVAL;
    }
    if (p->mode < MF4D_RIDGE || p->mode > MF4D_BOTH) return MF4D_EINVAL;
    if (!(p->lambda > 0.f)) return MF4D_EINVAL;   // +inf allowed, NaN rejected
    if (!(p->lambda * p->lambda > 0.f)) return MF4D_EINVAL;   // 1/lambda^2 must be finite
    if (!(p->rho >= 0.f) || !std::isfinite(p->rho) || (p->rho > 0.f && radius_of(p->rho) > kMaxRhoR))
        return MF4D_EINVAL;
    if (!(p->beta > 0.f) || !std::isfinite(p->beta)) return MF4D_EINVAL;
    if (!std::isfinite(p->c)) return MF4D_EINVAL;
    if (p->cycles < 0) return MF4D_EINVAL;
    if (!valid_tau_max(p->tau_max)) return MF4D_EINVAL;
    if (p->substeps < 0 || p->substeps > MF4D_MAX_SUBSTEPS) return MF4D_EINVAL;
    if (p->substeps == 0 && p->cycles > 0 && !(p->stop_time > 0.0 && std::isfinite(p->stop_time)))
        return MF4D_EINVAL;
    if (p->reselect_each_cycle != 0 && p->reselect_each_cycle != 1) return MF4D_EINVAL;
    if (p->postprocess != 0 && p->postprocess != 1) return MF4D_EINVAL;
    if (p->postprocess == 1 && !std::isfinite(p->theta)) return MF4D_EINVAL;
    if (p->check != 0 && p->check != 1) return MF4D_EINVAL;
    if (p->model != MF4D_MAFOD && p->model != MF4D_IFOD) return MF4D_EINVAL;
    if (p->model == MF4D_IFOD && p->nscales != 1) return MF4D_EINVAL;
    return MF4D_OK;
}

// Largest |partial product| of (1 - tau z) over z in {2q/(Q tau_max)}, q = 0..Q,
// over all prefixes and all suffixes of the ordered steps.
double partial_amplification(const std::vector<double> &ord, double tau_max)
{
    const int Q = 8192;
    const int n = (int)ord.size();
    double worst = 0.0;
    for (int q = 0; q <= Q; ++q) {
        const double z = 2.0 * (double)q / ((double)Q * tau_max);
        double acc = 1.0;
        for (int j = 0; j < n; ++j) {
            acc *= (1.0 - ord[j] * z);
            worst = std::fmax(worst, std::fabs(acc));
        }
        acc = 1.0;
        for (int j = n - 1; j >= 0; --j) {
            acc *= (1.0 - ord[j] * z);
            worst = std::fmax(worst, std::fabs(acc));
        }
    }
    return worst;
}

int gcd(int a, int b) { return b ? gcd(b, a % b) : a; }

// Orders the natural (ascending) steps as tau[(kappa j) mod n], with kappa the
// coprime multiplier of least partial amplification (ties -> smaller kappa).
int order_steps(const std::vector<double> &natural, double tau_max, double *out, int *perm)
{
    const int n = (int)natural.size();
    int kappa = 1;
    if (n > 2) {
        double best = INFINITY;
        std::vector<double> trial(n);
        for (int k = 1; k < n; ++k) {
            if (gcd(k, n) != 1) continue;
            for (int j = 0; j < n; ++j) trial[j] = natural[(int)(((long long)k * j) % n)];
            const double amp = partial_amplification(trial, tau_max);
            if (amp < best * (1.0 - 1e-12)) {
                best = amp;
                kappa = k;
            }
        }
    }
    for (int j = 0; j < n; ++j) {
        const int pj = (int)(((long long)kappa * j) % n);
        if (perm) perm[j] = pj;
        out[j] = natural[pj];
    }
    return kappa;
}

// Eq. (23) with cycle length T/M.
std::vector<double> natural_steps(int n, double T_over_M)
{
    std::vector<double> tau(n);
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < n; ++i) {
        const double c = std::cos(pi * (double)(2 * i + 1) / (double)(4 * n + 2));
        tau[i] = 3.0 * T_over_M / (2.0 * ((double)n * n + n) * c * c);
    }
    return tau;
}

struct Workspace {
    float *hA, *hB, *hC;     // horizontal pass, one scale at a time; then N at the chosen scale
    float *SA, *N;           // per-scale planes: (S, blob) pairs [ns][H][W][2], N [ns][H][W][3]
    uint8_t *idx;
    float *tens;             // compact tensor planes of the current cycle
    float *utmp;
    unsigned *smax;
    float *vmax;             // max_s V_s (postprocessing)
    uint8_t *idx2;           // postprocessed indices
    float *u2;               // second ping-pong image (l2-optimal stopping)
    double *partial;         // kRedBlocks partial sums of an l2 reduction
    MonitorState *mon;
};

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// one byte per 32 x 32 block (the learned filter's need bits)
size_t need_bytes(int H, int W) { return (size_t)((H + 31) / 32) * (size_t)((W + 31) / 32); }

size_t layout(int H, int W, int ns, Workspace *w, char *base)
{
    const size_t m = (size_t)H * W;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base ? base + off : nullptr;
        off += align256(bytes);
        return p;
    };
    Workspace t;
    t.hA = (float *)take(m * 12);
    t.hB = t.hA ? t.hA + m : nullptr;
    t.hC = t.hA ? t.hA + 2 * m : nullptr;
    t.SA = (float *)take(m * 8 * ns);
    t.N = (float *)take(m * 12 * ns);
    t.idx = (uint8_t *)take(m);
    t.tens = (float *)take(m * 12);
    t.utmp = (float *)take(m * 4);
    t.smax = (unsigned *)take(256);
    t.vmax = (float *)take(m * 4);
    t.idx2 = (uint8_t *)take(m);
    t.u2 = (float *)take(m * 4);
    t.partial = (double *)take(sizeof(double) * kRedBlocks);
    t.mon = (MonitorState *)take(sizeof(MonitorState));
    if (w) *w = t;
    return off;
}

int hip_status(hipError_t e) { return e == hipSuccess ? MF4D_OK : MF4D_EHIP; }

#define CHECK_HIP(expr)                              \
    do {                                             \
        hipError_t e_ = (expr);                      \
        if (e_ != hipSuccess) return MF4D_EHIP;      \
    } while (0)


// Rows per wave of the streaming substep kernel. Measured on MI355X at
// 4096 x 4096: ~96 rows for 3-4 substeps per launch, ~160 for 1-2; smaller
// images use shorter segments so that the grid still has ~4k waves.
// MF4D_STREAM_ROWS overrides (tuning).
int stream_rows(int H, int W, int steps)
{
    const char *e = std::getenv("MF4D_STREAM_ROWS");
    const int env = e ? std::atoi(e) : 0;
    if (env > 0) return env;
    // the longest segments (least row halo) whose waves still fit in one
    // round of resident blocks (with some slack, as blocks do not spread
    // perfectly evenly over the CUs); a partial second round would idle most
    // of the chip
    int cus = 256;
    const int per_cu = stream_blocks_per_cu(steps, &cus);
    const int cols = stream_cols_per_lane(steps);
    const int outw = 64 * cols - 4 * steps;
    const long long strips = (W + outw - 1) / outw;
    const long long waves = (4LL * per_cu * cus * 23) / 25;
    long long segs = waves / strips;
    if (segs < 1) segs = 1;
    int rows = (int)((H + segs - 1) / segs);
    // a wave walks rows + 4 steps rows in blocks of kStreamUnroll; a partial
    // last block is computed in full, so round to whole blocks: down, unless
    // that would overflow one round of resident blocks
    const int halo = 4 * steps;
    int r = ((rows + halo) / kStreamUnroll) * kStreamUnroll - halo;
    if (r < 16 || strips * ((H + r - 1) / r) > 4LL * per_cu * cus)
        r = ((rows + halo + kStreamUnroll - 1) / kStreamUnroll) * kStreamUnroll - halo;
    return r < 16 ? 16 : r;
}


// Side streams (default priority) and events for running independent
// launches concurrently with the caller's stream; one set per host thread and
// device, created on first use and kept until the process ends. MF4D_FORK=0
// turns the concurrency off.
constexpr int kForkStreams = 3;
struct ForkStreams {
    hipStream_t side[kForkStreams];
    hipEvent_t fork, join[kForkStreams];
};

ForkStreams *fork_streams()
{
    if (const char *e = std::getenv("MF4D_FORK"))
        if (std::atoi(e) == 0) return nullptr;
    thread_local ForkStreams *sets[16] = {};
    thread_local bool failed[16] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 16) return nullptr;
    if (sets[dev] || failed[dev]) return sets[dev];
    ForkStreams *f = new ForkStreams();
    bool ok = hipEventCreateWithFlags(&f->fork, hipEventDisableTiming) == hipSuccess;
    for (int i = 0; i < kForkStreams && ok; ++i)
        ok = hipStreamCreateWithFlags(&f->side[i], hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&f->join[i], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        failed[dev] = true;   // the caller's stream alone still works
        return nullptr;
    }
    sets[dev] = f;
    return f;
}

// Substeps of one cycle in launches of up to `spl` substeps.
int run_substeps(const float *u_first, float *const bufs[2], int &launch_index, const float *coef, int H,
                 int W, const float *tau32, int n, int spl, hipStream_t s, const float **last)
{
    const float *src = u_first;
    for (int i = 0; i < n;) {
        const int k = (n - i < spl) ? n - i : spl;
        float *dst = bufs[launch_index % 2];
        CHECK_HIP(launch_fed_stream(src, dst, coef, H, W, k, tau32 + i, stream_rows(H, W, k), s));
        ++launch_index;
        i += k;
        src = dst;
    }
    *last = src;
    return MF4D_OK;
}

// Scale sweep over all scales: S and blob planes (when want_sa), N planes
// (when want_n) and the image-wide maximum of S (cleared first unless
// clear_max is false: an earlier kernel on the stream has left it at 0).
int run_sweep(const float *u, int H, int W, const mf4d_params *p, const Workspace &w,
              bool want_n, hipStream_t s, bool clear_max = true, bool fork = true,
              const uint8_t *need = nullptr)
{
    const size_t m = (size_t)H * W;
    if (clear_max) CHECK_HIP(launch_fill_u32(w.smax, 0u, 1, s));
    std::vector<WinTaps> taps(p->nscales);
    bool fused = true;   // the fused kernels need no shared scratch: scales may run concurrently
    for (int k = 0; k < p->nscales; ++k) {
        make_taps(p->sigmas[k], &taps[k]);
        fused = fused && sweep_engine(taps[k]) == kSweepFused;
    }
    ForkStreams *fs = (fork && fused && p->nscales > 1) ? fork_streams() : nullptr;
    auto launch = [&](int k, hipStream_t st) {
        ScalePlanes planes{w.SA + 2 * k * m, want_n ? w.N + 3 * k * m : nullptr};
        return launch_sweep_scale(u, w.hA, w.hB, w.hC, H, W, taps[k], p->sigmas[k], p->mode, p->beta, planes,
                                  w.smax, fs != nullptr, st, ScaleNeed{need, (W + 31) / 32, k});
    };
    if (!fs) {
        for (int k = 0; k < p->nscales; ++k) CHECK_HIP(launch(k, s));
        return MF4D_OK;
    }
    // scales in the order largest, smallest, second largest, second smallest,
    // ..., spread round-robin over the caller's stream and the side streams,
    // so that each matrix-core bound large scale runs beside a memory-bound
    // small one (the scale index order is that of the sigmas)
    CHECK_HIP(hipEventRecord(fs->fork, s));
    for (int i = 0; i < kForkStreams; ++i) CHECK_HIP(hipStreamWaitEvent(fs->side[i], fs->fork, 0));
    for (int j = 0, lo = 0, hi = p->nscales - 1; j < p->nscales; ++j) {
        const int k = j % 2 == 0 ? hi-- : lo++;
        const int lane = j % (kForkStreams + 1);
        CHECK_HIP(launch(k, lane == 0 ? s : fs->side[lane - 1]));
    }
    for (int i = 0; i < kForkStreams; ++i) {
        CHECK_HIP(hipEventRecord(fs->join[i], fs->side[i]));
        CHECK_HIP(hipStreamWaitEvent(s, fs->join[i], 0));
    }
    return MF4D_OK;
}

SelectArgs select_args(const mf4d_params *p, const Workspace &w)
{
    SelectArgs a;
    std::memset(&a, 0, sizeof(a));
    a.SA = w.SA;
    a.N = w.N;
    a.ns = p->nscales;
    a.smax_bits = w.smax;
    a.c_param = p->c;
    a.mode = p->mode;
    a.inv_lam2 = 1.f / (p->lambda * p->lambda);
    make_rho_taps(p->rho, &a.rho);
    return a;
}

// Ordered schedules already computed, keyed by (n, T/M, tau_max) bit for bit:
// the kappa search costs O(phi(n) n Q) on the host, milliseconds at n = 10
// and a large fraction of a second at n in the hundreds, so every call after
// the first reuses it. The cache is bounded and shared by all threads.
struct Schedule {
    int n;
    double TM, tau_max;
    int kappa;
    std::vector<double> ordered;
    std::vector<int> perm;
};

const Schedule &cached_schedule(int n, double TM, double tau_max)
{
    static std::mutex mu;
    static std::vector<Schedule *> cache;
    std::lock_guard<std::mutex> lock(mu);
    for (const Schedule *c : cache)
        if (c->n == n && std::memcmp(&c->TM, &TM, sizeof TM) == 0 &&
            std::memcmp(&c->tau_max, &tau_max, sizeof tau_max) == 0)
            return *c;
    Schedule *c = new Schedule{n, TM, tau_max, 1, std::vector<double>(n), std::vector<int>(n)};
    c->kappa = order_steps(natural_steps(n, TM), tau_max, c->ordered.data(), c->perm.data());
    if (cache.size() >= 64) {   // entries stay valid for earlier callers: retire, do not free
        static std::vector<Schedule *> retired;
        retired.push_back(cache.front());
        cache.erase(cache.begin());
    }
    cache.push_back(c);
    return *c;
}

int plan(const mf4d_params *p, int *n_out, std::vector<double> &ordered)
{
    int n = p->substeps;
    double TM;
    if (n > 0) {
        TM = p->tau_max * ((double)n * n + n) / 3.0;
    } else {
        if (p->cycles < 1 || !(p->stop_time > 0.0)) return MF4D_EINVAL;
        n = mf4d_fed_substeps(p->stop_time, p->cycles, p->tau_max);
        if (n < 1) return MF4D_EINVAL;
        TM = p->stop_time / p->cycles;
    }
    ordered = cached_schedule(n, TM, p->tau_max).ordered;
    *n_out = n;
    return MF4D_OK;
}

// l2-optimal stopping (mf4d_filter_l2stop): the ground truth and the outputs.
struct StopArgs {
    const float *gt;
    double *l2_out;
    int *best_out;
};

float growth_tolerance()
{
    if (const char *e = std::getenv("MF4D_L2_GROWTH_TOL")) return (float)std::atof(e);
    return 1e-5f;
}

// Scale selection of one cycle into w.idx (raw argmax) or, with the
// postprocessing, w.idx2; returns the indices the tensor must use.
int select_cycle(const float *src, int H, int W, const mf4d_params *p, const Workspace &w, const SelectArgs &a,
                 bool first, bool reselect, hipStream_t s, bool fork)
{
    int st = run_sweep(src, H, W, p, w, true, s, first, fork);
    if (st != MF4D_OK) return st;
    SelectArgs ak = a;
    if (!p->postprocess) {
        if (reselect) ak.idx_out = w.idx;
        else ak.idx_in = w.idx;
        CHECK_HIP(launch_select(ak, H, W, s));
        return MF4D_OK;
    }
    if (reselect) {
        SelectArgs am = a;
        am.coef = nullptr;
        am.hrho = nullptr;
        am.smax_reset = nullptr;
        am.idx_out = w.idx;
        am.vmax_out = w.vmax;
        CHECK_HIP(launch_select(am, H, W, s));
        ScaleTable tab{};
        for (int k = 0; k < p->nscales; ++k) tab.s[k] = p->sigmas[k];
        const int tmax = (int)std::ceil(3.0 * (double)p->sigmas[p->nscales - 1]);
        CHECK_HIP(launch_postprocess(w.idx, w.vmax, w.N, p->nscales, H, W, tab, p->theta, tmax, w.idx2, s));
    }
    ak.idx_in = w.idx2;
    CHECK_HIP(launch_rho(ak, H, W, s));
    return MF4D_OK;
}

// Isotropic model: the tensor planes (g, 0, 0) of one cycle (and optionally
// the Hessian of u_sigma) from one horizontal pass and the g kernel.
int ifod_cycle(const float *src, int H, int W, const mf4d_params *p, const Workspace &w, float *coef, float *hess,
               hipStream_t s)
{
    WinTaps t;
    make_taps(p->sigmas[0], &t);
    CHECK_HIP(launch_hpass(src, w.hA, w.hB, w.hC, H, W, t, s));
    CHECK_HIP(launch_ifod_coef(w.hA, w.hB, w.hC, H, W, t, 1.f / (p->lambda * p->lambda), coef, hess, s));
    return MF4D_OK;
}

// The whole filter (a1-a7), optionally with the stability monitor
// (p->check) and l2-optimal stopping (stop != nullptr).
int run_filter(const float *u_in, float *u_out, int H, int W, const mf4d_params *p, char *base,
               const StopArgs *stop, hipStream_t s, bool fork = true)
{
    const size_t m = (size_t)H * W;
    Workspace w;
    layout(H, W, p->nscales, &w, base);
    const bool check = p->check == 1;
    const float tol = growth_tolerance();
    if (check || stop) CHECK_HIP(launch_monitor_reset(w.mon, s));
    if (check) CHECK_HIP(launch_l2(u_in, nullptr, m, w.partial, w.mon, kMonitorInit, tol, 0, nullptr, nullptr, s));
    if (stop) {
        CHECK_HIP(launch_l2(u_in, stop->gt, m, w.partial, w.mon, kStopStep, tol, 0, stop->l2_out, stop->best_out, s));
        CHECK_HIP(launch_copy_f32(u_in, u_out, m, s));
    }
    int st = MF4D_OK;
    if (p->cycles == 0) {
        if (!stop && u_in != u_out) CHECK_HIP(launch_copy_f32(u_in, u_out, m, s));
    } else {
        std::vector<double> ordered;
        int n = 0;
        st = plan(p, &n, ordered);
        if (st != MF4D_OK) return st;
        std::vector<float> tau32(n);
        for (int i = 0; i < n; ++i) tau32[i] = (float)ordered[i];
        // substeps run kSubstepsPerLaunch per launch (the intermediate images
        // stay in registers); the last launch of a cycle takes the remainder
        const int spl = kSubstepsPerLaunch;
        const int launches_per_cycle = (n + spl - 1) / spl;
        // launch j writes bufs[j % 2]; without stopping the last launch must
        // write u_out; with stopping the images ping-pong in the workspace and
        // the best one is copied to u_out
        const long long total = (long long)p->cycles * launches_per_cycle;
        float *bufs[2];
        const float *src = u_in;
        if (stop) {
            bufs[0] = w.utmp;
            bufs[1] = w.u2;
        } else {
            bufs[0] = (total % 2 == 1) ? u_out : w.utmp;
            bufs[1] = (total % 2 == 1) ? w.utmp : u_out;
            if ((const float *)bufs[0] == u_in) {
                // in-place call whose first launch would overwrite its own input
                CHECK_HIP(launch_copy_f32(u_in, w.utmp, m, s));
                src = w.utmp;
                bufs[0] = u_out;
                bufs[1] = w.utmp;
            }
        }
        SelectArgs a = select_args(p, w);
        a.coef = w.tens;
        a.smax_reset = w.smax;   // each cycle's integration clears the max of S for the next cycle's sweep
        int li = 0;
        for (int k = 0; k < p->cycles; ++k) {
            if (p->model == MF4D_IFOD) st = ifod_cycle(src, H, W, p, w, w.tens, nullptr, s);
            else st = select_cycle(src, H, W, p, w, a, k == 0, (k == 0) || p->reselect_each_cycle, s, fork);
            if (st != MF4D_OK) return st;
            st = run_substeps(src, bufs, li, w.tens, H, W, tau32.data(), n, spl, s, &src);
            if (st != MF4D_OK) return st;
            if (check)
                CHECK_HIP(launch_l2(src, nullptr, m, w.partial, w.mon, kMonitorCycle, tol, 0, nullptr, nullptr, s));
            if (stop) {
                CHECK_HIP(launch_l2(src, stop->gt, m, w.partial, w.mon, kStopStep, tol, k + 1, stop->l2_out,
                                    stop->best_out, s));
                CHECK_HIP(launch_take_copy(src, u_out, m, w.mon, s));
            }
        }
    }
    if (!check) return MF4D_OK;
    CHECK_HIP(hipStreamSynchronize(s));
    MonitorState h;
    CHECK_HIP(hipMemcpy(&h, w.mon, sizeof h, hipMemcpyDeviceToHost));
    if (h.nonfinite) return MF4D_ENONFINITE;
    if (h.growth) return MF4D_EUNSTABLE;
    return MF4D_OK;
}

// Scratch of mf4d_filter_noalloc: a file-scope device array, one per GPU,
// held from the library's first use on that GPU until the process ends. Host
// code never passes `scratch` itself to a kernel (on the host the name only
// stands in for the symbol): it uses the device address from
// hipGetSymbolAddress, taken once per device with that device current.
constexpr size_t kStaticScratchBytes = (size_t)128 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

char *static_scratch(int dev)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void *ptrs[kMaxDevices] = {};
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(mu);
    if (!ptrs[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
        ptrs[dev] = ptr;
    }
    return (char *)ptrs[dev];
}

}  // namespace

namespace mf4d {
// host helpers shared with the batch module (batch.hip)
int validate_params(int H, int W, const mf4d_params *p) { return validate(H, W, p); }
size_t image_workspace_bytes(int H, int W, int ns) { return layout(H, W, ns, nullptr, nullptr); }
void image_workspace(int H, int W, int ns, char *base, float **hA, float **SA, float **N,
                     uint8_t **idx, float **tens, float **utmp, unsigned **smax)
{
    Workspace w;
    layout(H, W, ns, &w, base);
    *hA = w.hA;
    *SA = w.SA;
    *N = w.N;
    *idx = w.idx;
    *tens = w.tens;
    *utmp = w.utmp;
    *smax = w.smax;
}
void window_taps(double sigma, WinTaps *t) { make_taps(sigma, t); }
void rho_taps(double rho, RhoTaps *t) { make_rho_taps(rho, t); }
int fed_plan_host(const mf4d_params *p, int *n_out, std::vector<double> &ordered) { return plan(p, n_out, ordered); }
int default_stream_rows(int H, int W, int steps) { return stream_rows(H, W, steps); }
}  // namespace mf4d

extern "C" {

const char *mf4d_status_string(int status)
{
    switch (status) {
    case MF4D_OK: return "ok";
    case MF4D_EINVAL: return "invalid argument";
    case MF4D_ENOMEM: return "workspace too small";
    case MF4D_EHIP: return "HIP runtime or launch error";
    case MF4D_ENONFINITE: return "non-finite value in the image";
    case MF4D_EUNSTABLE: return "l2 norm grew over a cycle";
    default: return "unknown status";
    }
}

int mf4d_params_default(mf4d_params *p, int nscales, const float *sigmas)
{
    if (!p) return MF4D_EINVAL;
    std::memset(p, 0, sizeof(*p));
    p->nscales = nscales;
    p->sigmas = sigmas;
    p->mode = MF4D_BOTH;
    p->lambda = 0.005f;
    p->rho = 0.5f;
    p->beta = 0.5f;
    p->c = -1.f;
    p->cycles = 1;
    p->substeps = 10;
    p->stop_time = 0.0;
    p->tau_max = 0.05;
    p->reselect_each_cycle = 1;
    p->theta = 0.f;
    p->postprocess = 0;
    return MF4D_OK;
}

int mf4d_fed_schedule(int n, double tau_max, double *taus_out, int *perm_out)
{
    if (n < 1 || n > MF4D_MAX_SUBSTEPS || !valid_tau_max(tau_max) || !taus_out) return MF4D_EINVAL;
    const double TM = tau_max * ((double)n * n + n) / 3.0;
    const Schedule &c = cached_schedule(n, TM, tau_max);
    std::memcpy(taus_out, c.ordered.data(), sizeof(double) * n);
    if (perm_out) std::memcpy(perm_out, c.perm.data(), sizeof(int) * n);
    return c.kappa;
}

int mf4d_fed_substeps(double stop_time, int cycles, double tau_max)
{
    if (!(stop_time > 0.0) || !std::isfinite(stop_time) || cycles < 1 || !valid_tau_max(tau_max))
        return MF4D_EINVAL;
    const double v = -0.5 + 0.5 * std::sqrt(1.0 + 12.0 * stop_time / ((double)cycles * tau_max));
    const double n = std::ceil(v);
    if (n < 1.0 || n > MF4D_MAX_SUBSTEPS) return MF4D_EINVAL;
    return (int)n;
}

int mf4d_fed_plan(const mf4d_params *p, int *n_out, double *taus_out)
{
    if (!p || !n_out || !valid_tau_max(p->tau_max)) return MF4D_EINVAL;
    std::vector<double> ord;
    int n = 0;
    int st = plan(p, &n, ord);
    if (st != MF4D_OK) return st;
    *n_out = n;
    if (taus_out) std::memcpy(taus_out, ord.data(), sizeof(double) * n);
    return MF4D_OK;
}

size_t mf4d_workspace_bytes(int H, int W, const mf4d_params *p)
{
    if (validate(H, W, p) != MF4D_OK) return 0;
    return layout(H, W, p->nscales, nullptr, nullptr);
}

int mf4d_scale_select(const float *u, int H, int W, const mf4d_params *p, uint8_t *idx_out,
                      float *vmax_out, float *c_out, void *ws, size_t ws_bytes, void *stream)
{
    int st = validate(H, W, p);
    if (st != MF4D_OK) return st;
    if (!u || !idx_out || !ws || p->model != MF4D_MAFOD) return MF4D_EINVAL;
    if (ws_bytes < layout(H, W, p->nscales, nullptr, nullptr)) return MF4D_ENOMEM;
    hipStream_t s = (hipStream_t)stream;
    Workspace w;
    layout(H, W, p->nscales, &w, (char *)ws);
    const bool post = p->postprocess == 1;
    st = run_sweep(u, H, W, p, w, post, s);   // the postprocessing reads the Hessians (N) of every scale
    if (st != MF4D_OK) return st;
    SelectArgs a = select_args(p, w);
    a.idx_out = post ? w.idx : idx_out;
    a.vmax_out = post ? w.vmax : vmax_out;
    a.c_out = c_out;
    CHECK_HIP(launch_select(a, H, W, s));
    if (!post) return MF4D_OK;
    ScaleTable tab{};
    for (int k = 0; k < p->nscales; ++k) tab.s[k] = p->sigmas[k];
    const int tmax = (int)std::ceil(3.0 * (double)p->sigmas[p->nscales - 1]);
    CHECK_HIP(launch_postprocess(w.idx, w.vmax, w.N, p->nscales, H, W, tab, p->theta, tmax, idx_out, s));
    if (vmax_out) CHECK_HIP(launch_copy_f32(w.vmax, vmax_out, (size_t)H * W, s));
    return MF4D_OK;
}

int mf4d_tensor(const float *u, int H, int W, const uint8_t *idx, const mf4d_params *p,
                float *hrho_out, float *dparams_out, void *ws, size_t ws_bytes, void *stream)
{
    int st = validate(H, W, p);
    if (st != MF4D_OK) return st;
    if (!u || !hrho_out || !ws || (!idx && p->model == MF4D_MAFOD)) return MF4D_EINVAL;
    if (ws_bytes < layout(H, W, p->nscales, nullptr, nullptr)) return MF4D_ENOMEM;
    hipStream_t s = (hipStream_t)stream;
    Workspace w;
    layout(H, W, p->nscales, &w, (char *)ws);
    if (p->model == MF4D_IFOD) return ifod_cycle(u, H, W, p, w, dparams_out ? dparams_out : w.tens, hrho_out, s);
    st = run_sweep(u, H, W, p, w, true, s);
    if (st != MF4D_OK) return st;
    SelectArgs a = select_args(p, w);
    a.idx_in = idx;
    a.hrho = hrho_out;
    a.coef = dparams_out;
    CHECK_HIP(launch_select(a, H, W, s));
    return MF4D_OK;
}

int mf4d_fed_cycle(float *u, float *u_tmp, int H, int W, const float *hrho, const mf4d_params *p,
                   const double *taus, int n, void *stream)
{
    int st = validate(H, W, p);
    if (st != MF4D_OK) return st;
    if (!u || !u_tmp || u == u_tmp || !hrho || !taus || n < 1 || n > MF4D_MAX_SUBSTEPS)
        return MF4D_EINVAL;
    if (p->model != MF4D_MAFOD) return MF4D_EINVAL;
    for (int i = 0; i < n; ++i)
        if (!(taus[i] > 0.0) || !std::isfinite(taus[i])) return MF4D_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const float inv_lam2 = 1.f / (p->lambda * p->lambda);
    float *src = u, *dst = u_tmp;
    for (int i = 0; i < n; ++i) {
        CHECK_HIP(launch_fed_substep(src, dst, hrho, H, W, (float)taus[i], p->mode, inv_lam2, s));
        float *t = src;
        src = dst;
        dst = t;
    }
    if (src != u) CHECK_HIP(launch_copy_f32(src, u, (size_t)H * W, s));
    return MF4D_OK;
}

int mf4d_fed_cycle_tensor(float *u, float *u_tmp, int H, int W, const float *dparams, const double *taus,
                          int n, int steps_per_launch, void *stream)
{
    if (H < 3 || W < 3 || (long long)H * (long long)W >= (1LL << 31)) return MF4D_EINVAL;
    if (!u || !u_tmp || u == u_tmp || !dparams || !taus || n < 1 || n > MF4D_MAX_SUBSTEPS)
        return MF4D_EINVAL;
    if (steps_per_launch < 1 || steps_per_launch > 4) return MF4D_EINVAL;
    for (int i = 0; i < n; ++i)
        if (!(taus[i] > 0.0) || !std::isfinite(taus[i])) return MF4D_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    std::vector<float> tau32(n);
    for (int i = 0; i < n; ++i) tau32[i] = (float)taus[i];
    float *const bufs[2] = {u_tmp, u};
    int li = 0;
    const float *last = nullptr;
    int st = run_substeps(u, bufs, li, dparams, H, W, tau32.data(), n, steps_per_launch, s, &last);
    if (st != MF4D_OK) return st;
    if (last != u) CHECK_HIP(launch_copy_f32(last, u, (size_t)H * W, s));
    return MF4D_OK;
}

int mf4d_filter(const float *u_in, float *u_out, int H, int W, const mf4d_params *p, void *ws,
                size_t ws_bytes, void *stream)
{
    int st = validate(H, W, p);
    if (st != MF4D_OK) return st;
    if (!u_in || !u_out || !ws) return MF4D_EINVAL;
    if (ws_bytes < layout(H, W, p->nscales, nullptr, nullptr)) return MF4D_ENOMEM;
    return run_filter(u_in, u_out, H, W, p, (char *)ws, nullptr, (hipStream_t)stream);
}

int mf4d_filter_noalloc(const float *u_in, float *u_out, int H, int W, const mf4d_params *p, void *stream)
{
    int st = validate(H, W, p);
    if (st != MF4D_OK) return st;
    if (!u_in || !u_out) return MF4D_EINVAL;
    if (layout(H, W, p->nscales, nullptr, nullptr) > kStaticScratchBytes) return MF4D_ENOMEM;
    int dev = -1;
    CHECK_HIP(hipGetDevice(&dev));
    char *base = static_scratch(dev);
    if (!base) return MF4D_EHIP;
    // every scale on the caller's stream: no side streams are created
    return run_filter(u_in, u_out, H, W, p, base, nullptr, (hipStream_t)stream, false);
}

size_t mf4d_noalloc_max_bytes(void) { return kStaticScratchBytes; }

int mf4d_filter_l2stop(const float *u_in, float *u_out, int H, int W, const mf4d_params *p,
                       const float *ground_truth, double *l2_out, int *best_out, void *ws, size_t ws_bytes,
                       void *stream)
{
    int st = validate(H, W, p);
    if (st != MF4D_OK) return st;
    if (!u_in || !u_out || !ground_truth || !ws || u_out == u_in || u_out == ground_truth) return MF4D_EINVAL;
    if (ws_bytes < layout(H, W, p->nscales, nullptr, nullptr)) return MF4D_ENOMEM;
    StopArgs stop{ground_truth, l2_out, best_out};
    return run_filter(u_in, u_out, H, W, p, (char *)ws, &stop, (hipStream_t)stream);
}

size_t mf4d_creases_workspace_bytes(int H, int W)
{
    if (H < 3 || W < 3 || (long long)H * (long long)W >= (1LL << 31)) return 0;
    const size_t m = (size_t)H * W;
    return align256(m * 12) + align256(m * 24);
}

int mf4d_creases(const float *u, int H, int W, float sigma_d, float strength, int mode, float *seg_out,
                 int8_t *type_out, unsigned *count_out, float *field_out, void *ws, size_t ws_bytes, void *stream)
{
    const size_t need = mf4d_creases_workspace_bytes(H, W);
    if (!need || !u || !seg_out || !type_out || !ws) return MF4D_EINVAL;
    if (!(sigma_d > 0.f) || !std::isfinite(sigma_d) || radius_of(sigma_d) > MF4D_MAX_RADIUS) return MF4D_EINVAL;
    if (!(strength >= 0.f) || !std::isfinite(strength)) return MF4D_EINVAL;
    if (mode < MF4D_RIDGE || mode > MF4D_BOTH) return MF4D_EINVAL;
    if (ws_bytes < need) return MF4D_ENOMEM;
    hipStream_t s = (hipStream_t)stream;
    const size_t m = (size_t)H * W;
    float *hA = (float *)ws;
    float *planes = field_out ? field_out : (float *)((char *)ws + align256(m * 12));
    WinTaps t;
    make_taps(sigma_d, &t);
    CHECK_HIP(launch_hpass(u, hA, hA + m, hA + 2 * m, H, W, t, s));
    CHECK_HIP(launch_crease_field(hA, hA + m, hA + 2 * m, H, W, t, planes, s));
    CHECK_HIP(launch_marching(planes, H, W, strength, mode, seg_out, type_out, count_out, s));
    return MF4D_OK;
}

int mf4d_crease_match(const float *seg, const int8_t *type, int H, int W, const float *gt, const int *gt_type, int n,
                      float radius, float *dist_out, int *match_out, void *stream)
{
    if (H < 3 || W < 3 || (long long)H * (long long)W >= (1LL << 31) || n < 0) return MF4D_EINVAL;
    if (!(radius >= 0.f) || !std::isfinite(radius)) return MF4D_EINVAL;
    if (n == 0) return MF4D_OK;
    if (!seg || !type || !gt || !gt_type || !dist_out || !match_out) return MF4D_EINVAL;
    CHECK_HIP(launch_crease_match(seg, type, H, W, gt, gt_type, n, radius, dist_out, match_out, (hipStream_t)stream));
    return MF4D_OK;
}

size_t mf4d_learned_workspace_bytes(int H, int W, const mf4d_params *p)
{
    if (validate(H, W, p) != MF4D_OK || p->nscales > 8 || H % 16 != 0 || W % 16 != 0) return 0;
    if (p->model != MF4D_MAFOD || p->postprocess != 0 || p->check != 0) return 0;
    return align256(layout(H, W, p->nscales, nullptr, nullptr)) + align256(net_forward_bytes(H, W)) +
           align256(sizeof(unsigned) * kFallbackSlots) + align256(need_bytes(H, W));
}

int mf4d_filter_learned(const float *u_in, float *u_out, int H, int W, const mf4d_params *p, const float *theta,
                        float conf_threshold, unsigned *fallback_count, void *ws, size_t ws_bytes, void *stream)
{
    int st = validate(H, W, p);
    if (st != MF4D_OK) return st;
    if (!u_in || !u_out || !theta || !ws || p->nscales > 8 || H % 16 != 0 || W % 16 != 0) return MF4D_EINVAL;
    if (!(conf_threshold >= 0.f) || conf_threshold > 1.f || p->reselect_each_cycle != 1) return MF4D_EINVAL;
    if (p->model != MF4D_MAFOD || p->postprocess != 0 || p->check != 0) return MF4D_EINVAL;
    if (ws_bytes < mf4d_learned_workspace_bytes(H, W, p)) return MF4D_ENOMEM;
    hipStream_t s = (hipStream_t)stream;
    const size_t m = (size_t)H * W;
    char *base = (char *)ws;
    const size_t img_bytes = align256(layout(H, W, p->nscales, nullptr, nullptr));
    char *net_ws = base + img_bytes;
    unsigned *fb = (unsigned *)(net_ws + align256(net_forward_bytes(H, W)));   // kFallbackSlots counters
    uint8_t *need = (uint8_t *)fb + align256(sizeof(unsigned) * kFallbackSlots);
    CHECK_HIP(launch_fill_u32(fb, 0u, kFallbackSlots, s));
    if (p->cycles == 0) {
        if (u_in != u_out) CHECK_HIP(launch_copy_f32(u_in, u_out, m, s));
        if (fallback_count) CHECK_HIP(launch_fallback_sum(fb, fallback_count, s));
        return MF4D_OK;
    }
    std::vector<double> ordered;
    int n = 0;
    st = plan(p, &n, ordered);
    if (st != MF4D_OK) return st;
    std::vector<float> tau32(n);
    for (int i = 0; i < n; ++i) tau32[i] = (float)ordered[i];
    const int spl = kSubstepsPerLaunch;
    const int launches_per_cycle = (n + spl - 1) / spl;
    Workspace w;
    layout(H, W, p->nscales, &w, base);
    const long long total = (long long)p->cycles * launches_per_cycle;
    float *bufs[2];
    bufs[0] = (total % 2 == 1) ? u_out : w.utmp;
    bufs[1] = (total % 2 == 1) ? w.utmp : u_out;
    const float *src = u_in;
    if ((const float *)bufs[0] == u_in) {
        CHECK_HIP(launch_copy_f32(u_in, w.utmp, m, s));
        src = w.utmp;
        bufs[0] = u_out;
        bufs[1] = w.utmp;
    }
    SelectArgs a = select_args(p, w);
    a.coef = w.tens;
    a.idx_out = w.idx;
    // the image-wide c of the first cycle, kept for the later ones (their
    // sweeps skip blocks where the network decides)
    unsigned *held = w.smax + 1;
    a.smax_bits = held;
    int li = 0;
    for (int k = 0; k < p->cycles; ++k) {
        const uint8_t *sel = nullptr;
        st = net_select_into(theta, src, H, W, net_ws, s, conf_threshold, p->nscales, &sel,
                             k == 0);   // weights packed once per call
        if (st != MF4D_OK) return st;
        if (k > 0) CHECK_HIP(launch_need_flags(sel, H, W, p->nscales, need, s));
        st = run_sweep(src, H, W, p, w, true, s, true, true, k > 0 ? need : nullptr);
        if (st != MF4D_OK) return st;
        if (k == 0) CHECK_HIP(launch_copy_f32((const float *)w.smax, (float *)held, 1, s));
        CHECK_HIP(launch_learned_select(sel, a, H, W, fb, s));
        CHECK_HIP(launch_rho(a, H, W, s));
        st = run_substeps(src, bufs, li, w.tens, H, W, tau32.data(), n, spl, s, &src);
        if (st != MF4D_OK) return st;
    }
    if (fallback_count) CHECK_HIP(launch_fallback_sum(fb, fallback_count, s));
    return MF4D_OK;
}

}  // extern "C"
