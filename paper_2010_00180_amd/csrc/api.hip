// Host side of the C ABI declared in include/ising_search.h: argument
// validation, device allocation, the per-step launch sequence and result
// copies.  Every device computation happens in the kernels (k_init.hip,
// k_step.hip, k_split.hip, k_learn.hip, k_mlp.hip); this file only moves data
// and orders launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "../../include/ising_search.h"
#include "bestfirst.h"
#include "common.h"

using namespace qi;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

constexpr uint32_t MAGIC = 0x51495331u;   // "QIS1"

// Live handles; a destroyed or foreign pointer is rejected without being read.
std::mutex g_live_mu;
std::set<const void*> g_live;

}  // namespace

struct ising_search {
    uint32_t magic = MAGIC;
    bool broken = false;
    ising_config_t cfg{};
    hipStream_t stream = nullptr;
    int device = 0;
    Layout lay{};
    std::vector<int> N;
    std::vector<int> Npad;
    int scan_grid = 0;
    bool final_dirty = true;
    std::vector<void*> allocs;
    uint64_t* x0 = nullptr;      // initial states, kept for reset
    // host mirrors of small device buffers
    int flags_h[8]{};
    // timing (cfg.timing): events around each kernel family of a step
    bool timing = false;
    hipEvent_t ev[8]{};
    double t_scan = 0, t_merge = 0, t_frontier = 0, t_prep = 0, t_init = 0, t_step = 0, t_learn = 0, t_bound = 0;
    // learned-proposal form
    bool scorer_set = false;
    bool record = false;
    bool tracing = false;
    int learn_grid = 0;
    float* d_mlp = nullptr;
    double split_err = 0;
    double* d_maxerr = nullptr;
    uint64_t scan_launches = 0;
    // states per scan item, per instance (host copy of lay.scb)
    std::vector<int> sc_h;
    int* d_scb = nullptr;
    bool sc_auto_ok = false;   // the configuration lets each step choose its states per item
    // persistent mode: one step captured into a graph
    bool persistent = false;
    hipStream_t own_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    // tuned scan tiles: cache file (empty = none) and the device's architecture
    std::string tile_cache;
    std::string arch;
    // run() in persistent mode: graph_steps steps captured into one graph
    int graph_steps = 1;
    hipGraph_t graph_k = nullptr;
    hipGraphExec_t gexec_k = nullptr;
};

namespace {

#define HIP_TRY(expr)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess) {                                                           \
            return fail(ISING_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));   \
        }                                                                                 \
    } while (0)

template <class T>
int dalloc(ising_search* h, T** p, size_t count)
{
    void* v = nullptr;
    size_t bytes = count * sizeof(T);
    if (bytes == 0) bytes = 8;
    hipError_t e = hipMalloc(&v, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(ISING_ERR_OUT_OF_MEMORY, "hipMalloc of %zu bytes failed: %s", bytes, hipGetErrorString(e));
    }
    h->allocs.push_back(v);
    *p = static_cast<T*>(v);
    return ISING_OK;
}

void free_all(ising_search* h)
{
    if (h->gexec_k) (void)hipGraphExecDestroy(h->gexec_k);
    if (h->graph_k) (void)hipGraphDestroy(h->graph_k);
    h->gexec_k = nullptr;
    h->graph_k = nullptr;
    if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    h->gexec = nullptr;
    h->graph = nullptr;
    for (void* p : h->allocs) (void)hipFree(p);
    h->allocs.clear();
    if (h->own_stream) (void)hipStreamDestroy(h->own_stream);
    h->own_stream = nullptr;
    for (hipEvent_t& e : h->ev) {
        if (e) (void)hipEventDestroy(e);
        e = nullptr;
    }
}

// The captured step holds the Layout by value: drop it when the layout changes.
void drop_graph(ising_search* h)
{
    if (h->gexec_k) (void)hipGraphExecDestroy(h->gexec_k);
    if (h->graph_k) (void)hipGraphDestroy(h->graph_k);
    h->gexec_k = nullptr;
    h->graph_k = nullptr;
    if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    h->gexec = nullptr;
    h->graph = nullptr;
}

float elapsed_ms(hipEvent_t a, hipEvent_t b)
{
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) {
        (void)hipGetLastError();
        return 0.f;
    }
    return ms;
}

uint64_t splitmix64(uint64_t& x)
{
    uint64_t z = (x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

bool on_grid(double v)
{
    if (!std::isfinite(v)) return false;
    const double s = v * 16777216.0;   // 2^24
    if (std::fabs(s) > 9.0e15) return false;
    return s == std::nearbyint(s);
}

int check_handle(ising_search_t* s)
{
    if (!s) return fail(ISING_ERR_BAD_STATE, "NULL handle");
    {
        std::lock_guard<std::mutex> g(g_live_mu);
        if (!g_live.count(s)) return fail(ISING_ERR_BAD_STATE, "handle is not live (destroyed or never created)");
    }
    if (s->magic != MAGIC) return fail(ISING_ERR_BAD_STATE, "handle is corrupt");
    if (s->broken) return fail(ISING_ERR_BAD_STATE, "handle is unusable after an earlier device error");
    return ISING_OK;
}

// The network's parameter vector from a file of MLP_NPARAM little-endian
// FP32 values.
int read_weights(const char* path, std::vector<float>& out)
{
    FILE* f = std::fopen(path, "rb");
    if (!f) return fail(ISING_ERR_INVALID_ARG, "mlp_weights %s cannot be read", path);
    std::vector<unsigned char> raw(sizeof(float) * MLP_NPARAM + 1);
    const size_t got = std::fread(raw.data(), 1, raw.size(), f);
    std::fclose(f);
    if (got != sizeof(float) * MLP_NPARAM)
        return fail(ISING_ERR_INVALID_ARG, "mlp_weights %s: %zu bytes, expected %zu (%d FP32 values)", path, got,
                    sizeof(float) * MLP_NPARAM, MLP_NPARAM);
    out.assign(MLP_NPARAM, 0.f);
    for (int k = 0; k < MLP_NPARAM; ++k) {
        const unsigned char* b = raw.data() + 4 * k;
        const uint32_t u = (uint32_t)b[0] | ((uint32_t)b[1] << 8) | ((uint32_t)b[2] << 16) | ((uint32_t)b[3] << 24);
        std::memcpy(&out[k], &u, 4);
        if (!std::isfinite(out[k])) return fail(ISING_ERR_INVALID_ARG, "mlp_weights %s: value %d is not finite", path, k);
    }
    return ISING_OK;
}

// Tile cache lines: "ising-tile 1 <arch> <form> <flags> <N> <M> <states per item> <per-step>".
struct TileKey {
    std::string arch;
    int form, flags, N, M;
};

void read_tile_cache(const std::string& path, const TileKey& k, int& spi, int& per_step)
{
    spi = 0;
    per_step = 0;
    FILE* f = std::fopen(path.c_str(), "r");
    if (!f) return;
    char line[512];
    while (std::fgets(line, sizeof line, f)) {
        char tag[32], arch[256];
        int ver, form, flags, N, M, v, a;
        if (std::sscanf(line, "%31s %d %255s %d %d %d %d %d %d", tag, &ver, arch, &form, &flags, &N, &M, &v, &a) != 9)
            continue;
        if (std::strcmp(tag, "ising-tile") != 0 || ver != 1) continue;
        if (k.arch != arch || k.form != form || k.flags != flags || k.N != N || k.M != M) continue;
        if (v != 16 && v != 32 && v != 64 && v != 128 && v != 256) continue;
        spi = v;   // the last matching line wins
        per_step = a != 0;
    }
    std::fclose(f);
}

int append_tile_cache(const std::string& path, const TileKey& k, int spi, int per_step)
{
    FILE* f = std::fopen(path.c_str(), "a");
    if (!f) return fail(ISING_ERR_INVALID_ARG, "tile_cache %s cannot be opened to append", path.c_str());
    std::fprintf(f, "ising-tile 1 %s %d %d %d %d %d %d\n", k.arch.c_str(), k.form, k.flags, k.N, k.M, spi, per_step);
    const bool ok = std::fclose(f) == 0;
    return ok ? ISING_OK : fail(ISING_ERR_INVALID_ARG, "tile_cache %s could not be written", path.c_str());
}

int sync_flags(ising_search* h)
{
    HIP_TRY(hipMemcpyAsync(h->flags_h, h->lay.flags, sizeof(h->flags_h), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return ISING_OK;
}

}  // namespace

extern "C" const char* ising_search_last_error(void) { return g_err.c_str(); }

extern "C" int ising_search_init(ising_search_t** out, const ising_config_t* cfg, int32_t n_inst,
                                 const int32_t* N, const double* const* J, const double* const* h,
                                 int32_t L, const uint64_t* const* init_bits, void* stream)
{
    g_err.clear();
    if (!out) return fail(ISING_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!cfg) return fail(ISING_ERR_INVALID_ARG, "cfg is NULL");
    if (cfg->M < 1 || cfg->M > 1024) return fail(ISING_ERR_INVALID_ARG, "M=%d outside [1, 1024]", cfg->M);
    if (cfg->form != ISING_FORM_PLAIN && cfg->form != ISING_FORM_SPLIT_BF16 && cfg->form != ISING_FORM_LEARNED)
        return fail(ISING_ERR_INVALID_ARG, "form %d is unknown (0 plain, 1 split-bf16, 2 learned)", cfg->form);
    if (cfg->flags & ~(ISING_FLAG_RECORD_PROPOSALS | ISING_FLAG_SITE_BOUND | ISING_FLAG_FP16_SCAN |
                       ISING_FLAG_SINGLE_FLIPS | ISING_FLAG_EXCHANGE))
        return fail(ISING_ERR_INVALID_ARG, "unknown flag bits 0x%x", cfg->flags);
    const bool h1_singles = (cfg->flags & ISING_FLAG_SINGLE_FLIPS) != 0;
    const bool h1_exchange = (cfg->flags & ISING_FLAG_EXCHANGE) != 0;
    if (h1_singles && h1_exchange)
        return fail(ISING_ERR_INVALID_ARG, "single flips and exchanges are two different choices of H1");
    if ((h1_singles || h1_exchange) && cfg->form != ISING_FORM_PLAIN)
        return fail(ISING_ERR_INVALID_ARG, "the single-flip and exchange neighbourhoods run in the plain form only");
    if (h1_singles && (cfg->flags & ISING_FLAG_SITE_BOUND))
        return fail(ISING_ERR_INVALID_ARG, "the site bound skips pair flips, which the single-flip neighbourhood has none of");
    if ((cfg->flags & ISING_FLAG_FP16_SCAN) && cfg->form != ISING_FORM_SPLIT_BF16)
        return fail(ISING_ERR_INVALID_ARG, "the FP16 scan belongs to the split form");
    if ((cfg->flags & ISING_FLAG_RECORD_PROPOSALS) && cfg->form != ISING_FORM_LEARNED)
        return fail(ISING_ERR_INVALID_ARG, "proposals are recorded by the learned form only");
    if ((cfg->flags & ISING_FLAG_SITE_BOUND) && cfg->form == ISING_FORM_LEARNED)
        return fail(ISING_ERR_INVALID_ARG, "the site bound is available for the plain and split forms only");
    if (cfg->topk_factor < 0 || cfg->topk_factor > 64)
        return fail(ISING_ERR_INVALID_ARG, "topk_factor=%d outside [0, 64]", cfg->topk_factor);
    if (cfg->graph_steps < 0 || cfg->graph_steps > MAX_GRAPH_STEPS)
        return fail(ISING_ERR_INVALID_ARG, "graph_steps=%d outside [0, %d]", cfg->graph_steps, MAX_GRAPH_STEPS);
    if (cfg->surv_capacity != 0 && (cfg->surv_capacity < 2 * cfg->M || cfg->surv_capacity < 64 ||
                                    cfg->surv_capacity > MAX_SURV_CAP))
        return fail(ISING_ERR_INVALID_ARG, "surv_capacity=%d: 0, or between max(2M, 64) and 2^24", cfg->surv_capacity);
    int rc0 = ISING_OK;
    if (cfg->states_per_item < 0 || cfg->states_per_item > 4096)
        return fail(ISING_ERR_INVALID_ARG, "states_per_item=%d outside [0, 4096]", cfg->states_per_item);
    std::vector<float> weights;
    if (cfg->mlp_weights) {
        if (cfg->form != ISING_FORM_LEARNED)
            return fail(ISING_ERR_INVALID_ARG, "mlp_weights belongs to the learned form");
        rc0 = read_weights(cfg->mlp_weights, weights);
        if (rc0 != ISING_OK) return rc0;
    }
    if (cfg->tile_cache && cfg->tile_cache[0]) {
        FILE* f = std::fopen(cfg->tile_cache, "a");
        if (!f) return fail(ISING_ERR_INVALID_ARG, "tile_cache %s cannot be opened to append", cfg->tile_cache);
        std::fclose(f);
    }
    if (n_inst < 1) return fail(ISING_ERR_INVALID_ARG, "n_inst=%d < 1", n_inst);
    if (L < 1) return fail(ISING_ERR_INVALID_ARG, "L=%d < 1", L);
    if (!N || !J || !h || !init_bits) return fail(ISING_ERR_INVALID_ARG, "NULL array argument");
    if ((long long)n_inst * L > (1 << 24)) return fail(ISING_ERR_INVALID_ARG, "too many searches");

    int Nmax = 0;
    bool j32_exact = true;   // every 4J_ij exactly representable in FP32
    // local fields as 32-bit integers: instance b's grid 2^-g_b (the coarsest
    // power of two that all its values are multiples of, g_b in [0, 24]) and
    // |F_i| <= |h_i| + sum_j |J_ij| < 2^31 grid units for every instance
    bool fq_ok = true;
    std::vector<int> fgrid(n_inst, 0);
    for (int b = 0; b < n_inst; ++b) {
        if (N[b] < 1 || N[b] > MAX_N) return fail(ISING_ERR_INVALID_ARG, "N[%d]=%d outside [1, %d]", b, N[b], MAX_N);
        if (!J[b] || !h[b] || !init_bits[b]) return fail(ISING_ERR_INVALID_ARG, "NULL pointer for instance %d", b);
        if (N[b] > Nmax) Nmax = N[b];
        const int n = N[b];
        double bound = 0.0;
        std::vector<double> row(n, 0.0);
        int tz = 24;   // fewest trailing zero bits of a value in units of 2^-24
        auto grid_of = [&](double v) {
            const long long t = std::llabs((long long)(v * 16777216.0));
            if (t != 0) tz = std::min(tz, __builtin_ctzll((unsigned long long)t));
        };
        for (int i = 0; i < n; ++i) {
            if (!on_grid(h[b][i]))
                return fail(ISING_ERR_INVALID_ARG, "h[%d][%d]=%g is not a finite multiple of 2^-24", b, i, h[b][i]);
            bound += std::fabs(h[b][i]);
            row[i] += std::fabs(h[b][i]);
            grid_of(h[b][i]);
            if (J[b][(size_t)i * n + i] != 0.0)
                return fail(ISING_ERR_INVALID_ARG, "J[%d] has a nonzero diagonal at %d", b, i);
            for (int j = i + 1; j < n; ++j) {
                const double v = J[b][(size_t)i * n + j];
                if (!on_grid(v))
                    return fail(ISING_ERR_INVALID_ARG, "J[%d][%d,%d]=%g is not a finite multiple of 2^-24", b, i, j, v);
                if (v != J[b][(size_t)j * n + i])
                    return fail(ISING_ERR_INVALID_ARG, "J[%d] is not symmetric at (%d,%d)", b, i, j);
                if ((double)(float)(4.0 * v) != 4.0 * v) j32_exact = false;
                bound += std::fabs(v);
                row[i] += std::fabs(v);
                row[j] += std::fabs(v);
                grid_of(v);
            }
        }
        if (bound > 16777216.0)
            return fail(ISING_ERR_INVALID_ARG, "instance %d: sum |J_ij| + sum |h_i| = %g exceeds 2^24", b, bound);
        fgrid[b] = 24 - tz;
        const double rmax = *std::max_element(row.begin(), row.end());
        if (!(std::ldexp(rmax, fgrid[b]) < 2147483648.0)) fq_ok = false;
        const int W = words_of(n);
        int downs0 = -1;
        for (int l = 0; l < L; ++l) {
            const uint64_t* x = init_bits[b] + (size_t)l * W;
            const int tail = n & 63;
            if (tail && (x[W - 1] >> tail))
                return fail(ISING_ERR_INVALID_ARG, "initial state %d of instance %d has bits at positions >= N", l, b);
            int downs = 0;
            for (int w = 0; w < W; ++w) downs += __builtin_popcountll(x[w]);
            if (h1_exchange && downs0 >= 0 && downs != downs0)
                return fail(ISING_ERR_INVALID_ARG, "exchanges conserve the number of down spins: the initial states of "
                            "instance %d lie in different sectors (%d and %d down spins)", b, downs0, downs);
            downs0 = downs;
        }
    }

    // learned form: K = topk * N proposals per state; candidate keys in LDS are
    // twice K when two blocks still fit a CU, else as many as one block may
    // hold, and at least K plus one round of appends
    const int topk = cfg->topk_factor > 0 ? cfg->topk_factor : 8;
    int kmax = 1, cap_lr = 0;
    {
        const long long allp = (long long)Nmax * (Nmax - 1) / 2;
        const long long k = (long long)topk * Nmax;
        kmax = (int)std::max(1LL, std::min(k, allp));
    }
    if (cfg->form == ISING_FORM_LEARNED) {
        const long long fixed = (long long)words_of(Nmax) * 8 + (long long)pad_of(Nmax) * 2 + 2048;
        const long long want = 2LL * kmax + 1024;
        const long long room = LR_ROOM;
        long long cap = want;
        if (cap * 8 + fixed > 78 * 1024) {
            const long long two = (78 * 1024 - fixed) / 8;
            cap = two >= kmax + 2 * room ? two : std::min(want, (150 * 1024 - fixed) / 8);
        }
        if (cap < kmax + room)
            return fail(ISING_ERR_INVALID_ARG, "K = %d proposals per state do not fit the ranking kernel's LDS "
                        "(use a smaller topk_factor)", kmax);
        cap_lr = (int)cap;
    }

    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        return fail(ISING_ERR_NO_DEVICE, "no HIP device available");
    }

    ising_search* hd = new ising_search();
    hd->cfg = *cfg;
    if (hd->cfg.max_iters <= 0) hd->cfg.max_iters = 4 * Nmax + 16;
    hd->stream = static_cast<hipStream_t>(stream);
    if (hipGetDevice(&hd->device) != hipSuccess) {
        delete hd;
        return fail(ISING_ERR_HIP, "hipGetDevice failed");
    }
    Layout& lay = hd->lay;
    lay.B = n_inst;
    lay.L = L;
    lay.M = cfg->M;
    lay.S = n_inst * L;
    lay.Wmax = words_of(Nmax);
    lay.Npmax = pad_of(Nmax);
    lay.fmax = L * cfg->M;
    lay.cap_surv = cfg->surv_capacity > 0 ? cfg->surv_capacity : (cfg->form == ISING_FORM_LEARNED ? 65536 : 32768);
    lay.topk = topk;
    lay.kmax = kmax;
    lay.cap_lr = cap_lr;
    hd->record = (cfg->flags & ISING_FLAG_RECORD_PROPOSALS) != 0;
    const int sc0 = cfg->states_per_item > 0 ? cfg->states_per_item : 64;
    hd->sc_h.assign(n_inst, sc0);
    hd->persistent = cfg->persistent != 0;
    hd->graph_steps = hd->persistent ? (cfg->graph_steps > 0 ? cfg->graph_steps : 8) : 1;
    if (hd->persistent && !hd->stream) {
        // a graph cannot be captured on the legacy default stream
        if (hipStreamCreateWithFlags(&hd->own_stream, hipStreamNonBlocking) != hipSuccess) {
            delete hd;
            return fail(ISING_ERR_HIP, "hipStreamCreate failed");
        }
        hd->stream = hd->own_stream;
    }
    hd->N.assign(N, N + n_inst);
    hd->Npad.resize(n_inst);
    std::vector<long long> joff(n_inst);
    long long jtot = 0;
    for (int b = 0; b < n_inst; ++b) {
        hd->Npad[b] = pad_of(N[b]);
        joff[b] = jtot;
        jtot += (long long)hd->Npad[b] * hd->Npad[b];
    }

    int rc = ISING_OK;
    int *dN = nullptr, *dNpad = nullptr;
    long long* djoff = nullptr;
    double *dJ4 = nullptr, *dh = nullptr;
    uint64_t *dz = nullptr, *dx0 = nullptr;
    const size_t S = lay.S, M2 = 2 * (size_t)lay.M;
#define ALLOC(p, n) \
    if (rc == ISING_OK) rc = dalloc(hd, &(p), (n))
    ALLOC(dN, n_inst);
    ALLOC(dNpad, n_inst);
    ALLOC(djoff, n_inst);
    ALLOC(dJ4, (size_t)jtot);
    ALLOC(dh, (size_t)n_inst * lay.Npmax);
    ALLOC(dz, (size_t)MAX_N);
    ALLOC(dx0, S * lay.Wmax);
    ALLOC(lay.bits, S * M2 * lay.Wmax);
    ALLOC(lay.E, S * M2);
    ALLOC(lay.zob, S * M2);
    if (fq_ok) {
        ALLOC(lay.Fq, S * M2 * lay.Npmax);
    } else {
        ALLOC(lay.Fd, S * M2 * lay.Npmax);
    }
    double* dfsc = nullptr;
    ALLOC(dfsc, n_inst);
    ALLOC(lay.fresh, S * M2);
    ALLOC(lay.kept, S * lay.M);
    ALLOC(lay.nkept, S);
    ALLOC(lay.active, S);
    ALLOC(lay.retry, S);
    ALLOC(lay.cut, S);
    ALLOC(lay.fr_count, n_inst);
    ALLOC(lay.fr_list, (size_t)n_inst * lay.fmax);
    ALLOC(lay.A, (size_t)n_inst * lay.fmax * lay.Npmax);
    ALLOC(lay.rec, (size_t)n_inst * lay.fmax);
    ALLOC(lay.fbits, (size_t)n_inst * lay.fmax * lay.Wmax);
    ALLOC(lay.surv_count, S);
    ALLOC(lay.surv, S * lay.cap_surv);
    ALLOC(lay.item_prefix, 4 * ((size_t)n_inst + 1));
    ALLOC(lay.ctr, 16);
    ALLOC(lay.flags, 8);
    ALLOC(lay.step_active, MAX_GRAPH_STEPS);
    ALLOC(hd->d_scb, n_inst);
    float* dJ32 = nullptr;
    uint16_t *dJhi = nullptr, *dJlo = nullptr;
    double *dyb = nullptr, *debf = nullptr, *dab = nullptr;
    const bool need_j32 = cfg->form == ISING_FORM_SPLIT_BF16 || j32_exact;
    if (need_j32) ALLOC(dJ32, (size_t)jtot);
    const bool h16 = (cfg->flags & ISING_FLAG_FP16_SCAN) != 0;
    uint16_t* dJ16 = nullptr;
    if (h16) ALLOC(dJ16, (size_t)jtot);
    if (cfg->form == ISING_FORM_SPLIT_BF16) {
        ALLOC(dJhi, (size_t)jtot);
        ALLOC(dJlo, (size_t)jtot);
        ALLOC(dyb, n_inst);
        ALLOC(debf, n_inst);
        ALLOC(dab, n_inst);
        ALLOC(lay.Ft, S * lay.Npmax);
        ALLOC(lay.A32, (size_t)n_inst * lay.fmax * lay.Npmax);
        ALLOC(lay.RR32, (size_t)n_inst * lay.fmax * lay.Npmax);
        ALLOC(hd->d_maxerr, 1);
    }
    uint16_t* dJn = nullptr;
    if (cfg->form == ISING_FORM_LEARNED) {
        ALLOC(lay.xfull, S * M2);
        ALLOC(lay.mode, S);
        ALLOC(lay.last_mode, S);
        ALLOC(dJn, (size_t)jtot);
        ALLOC(hd->d_mlp, (size_t)MLP_NPARAM);
        if (hd->record) {
            ALLOC(lay.prop, (size_t)n_inst * lay.fmax * lay.kmax);
            ALLOC(lay.prop_n, (size_t)n_inst * lay.fmax);
        }
    }
    const bool sb = (cfg->flags & ISING_FLAG_SITE_BOUND) != 0;
    float* drm = nullptr;
    if (sb) {
        ALLOC(drm, (size_t)n_inst * lay.Npmax);
        ALLOC(lay.fr_bound, (size_t)n_inst * lay.fmax);
        ALLOC(lay.full_list, (size_t)n_inst * lay.fmax);
        ALLOC(lay.full_count, n_inst);
    }
    ALLOC(lay.lr_count, n_inst);
    ALLOC(lay.nm_count, S);
    ALLOC(lay.nm_code, S * lay.M);
    ALLOC(lay.nm_pair, S * lay.M);
    ALLOC(lay.nm_slot, S * lay.M);
    ALLOC(lay.out_bits, (size_t)n_inst * lay.M * lay.Wmax);
    ALLOC(lay.out_E, (size_t)n_inst * lay.M);
    ALLOC(lay.out_count, n_inst);
#undef ALLOC
    if (rc != ISING_OK) {
        free_all(hd);
        delete hd;
        return rc;
    }
    lay.N = dN;
    lay.Npad = dNpad;
    lay.joff = djoff;
    lay.J4 = dJ4;
    lay.h = dh;
    lay.zkey = dz;
    lay.scb = hd->d_scb;
    lay.form = cfg->form;
    lay.J32 = dJ32;
    lay.J4f = j32_exact ? dJ32 : nullptr;
    lay.Jhi = dJhi;
    lay.Jlo = dJlo;
    lay.ybound = dyb;
    lay.ebf = debf;
    lay.abound = dab;
    lay.Jn16 = dJn;
    lay.sb = sb ? 1 : 0;
    lay.h16 = h16 ? 1 : 0;
    lay.h1 = h1_singles ? H1_SINGLES : (h1_exchange ? H1_EXCHANGE : H1_FLIPS);
    // states per scan item chosen each step unless given, tuned, or the scan
    // serves only the states the site bound leaves (or ranked ones)
    lay.sc_auto = (cfg->states_per_item == 0 && !sb && cfg->form != ISING_FORM_LEARNED) ? 1 : 0;
    hd->sc_auto_ok = lay.sc_auto != 0;
    lay.J16 = dJ16;
    lay.rmax4 = drm;
    lay.fsc = dfsc;
    lay.mlp = hd->d_mlp;
    lay.scorer = 0;
    lay.seed = 0;
    hd->x0 = dx0;
    hd->timing = cfg->timing != 0;
    if (hd->timing) {
        for (hipEvent_t& e : hd->ev) {
            if (hipEventCreate(&e) != hipSuccess) {
                free_all(hd);
                delete hd;
                return fail(ISING_ERR_HIP, "hipEventCreate failed");
            }
        }
    }

    // host staging of padded 4J and h
    auto bail = [&](int code) {
        free_all(hd);
        delete hd;
        return code;
    };
    {
        std::vector<double> J4h((size_t)jtot, 0.0);
        std::vector<double> hh((size_t)n_inst * lay.Npmax, 0.0);
        std::vector<uint64_t> x0((size_t)S * lay.Wmax, 0);
        for (int b = 0; b < n_inst; ++b) {
            const int n = N[b], np = hd->Npad[b];
            double* dst = J4h.data() + joff[b];
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) dst[(size_t)i * np + j] = 4.0 * J[b][(size_t)i * n + j];
            for (int i = 0; i < n; ++i) hh[(size_t)b * lay.Npmax + i] = h[b][i];
            const int W = words_of(n);
            for (int l = 0; l < L; ++l)
                for (int w = 0; w < W; ++w)
                    x0[((size_t)b * L + l) * lay.Wmax + w] = init_bits[b][(size_t)l * W + w];
        }
        std::vector<uint64_t> zk(MAX_N);
        uint64_t st = 0x2010001800000001ull;
        for (auto& z : zk) z = splitmix64(st);
        const hipStream_t sm = hd->stream;
        int r2 = ISING_OK;
        auto cp = [&](void* d, const void* src, size_t bytes) {
            if (r2 != ISING_OK) return;
            hipError_t e = hipMemcpyAsync(d, src, bytes, hipMemcpyHostToDevice, sm);
            if (e != hipSuccess) r2 = fail(ISING_ERR_HIP, "host-to-device copy failed: %s", hipGetErrorString(e));
        };
        cp(dN, N, sizeof(int) * n_inst);
        cp(dNpad, hd->Npad.data(), sizeof(int) * n_inst);
        cp(djoff, joff.data(), sizeof(long long) * n_inst);
        cp(dJ4, J4h.data(), sizeof(double) * J4h.size());
        cp(dh, hh.data(), sizeof(double) * hh.size());
        cp(dz, zk.data(), sizeof(uint64_t) * zk.size());
        cp(dx0, x0.data(), sizeof(uint64_t) * x0.size());
        cp(hd->d_scb, hd->sc_h.data(), sizeof(int) * n_inst);
        std::vector<float> J32h;
        std::vector<uint16_t> hih, loh;
        if (need_j32) {
            // fl32(4J): the FP32 scan's couplings, and an exact copy when j32_exact
            J32h.assign((size_t)jtot, 0.f);
            for (int b = 0; b < n_inst; ++b) {
                const int n = N[b], np = hd->Npad[b];
                for (int i = 0; i < n; ++i)
                    for (int j = 0; j < n; ++j)
                        J32h[joff[b] + (size_t)i * np + j] = (float)(4.0 * J[b][(size_t)i * n + j]);
            }
            cp(dJ32, J32h.data(), sizeof(float) * J32h.size());
        }
        std::vector<double> ybh, ebfh, abh;
        if (cfg->form == ISING_FORM_SPLIT_BF16) {
            // fl32(4J), bf16 hi = RN(4J), lo = RN(4J - hi); per instance max |4J| and the
            // bound on |F~ - F|: split residual |4J - hi - lo| <= 2^-15 |4J| (two roundings to 8
            // significant bits, with margin for the float step), FP32 accumulation of 2N terms
            // <= 2.1 N 2^-24 sum|terms|, and the final FP32 add.
            auto bf16_rn = [](float f) -> uint16_t {
                uint32_t u;
                std::memcpy(&u, &f, 4);
                u += 0x7FFFu + ((u >> 16) & 1u);
                return (uint16_t)(u >> 16);
            };
            auto bf16_to_f = [](uint16_t b) -> float {
                const uint32_t u = (uint32_t)b << 16;
                float f;
                std::memcpy(&f, &u, 4);
                return f;
            };
            hih.assign((size_t)jtot, 0);
            loh.assign((size_t)jtot, 0);
            ybh.assign(n_inst, 0.0);
            ebfh.assign(n_inst, 0.0);
            abh.assign(n_inst, 0.0);
            for (int b = 0; b < n_inst; ++b) {
                const int n = N[b], np = hd->Npad[b];
                double emax = 0.0;
                for (int i = 0; i < n; ++i) {
                    double R = 0.0;
                    for (int j = 0; j < n; ++j) {
                        const double x = 4.0 * J[b][(size_t)i * n + j];
                        const size_t o = joff[b] + (size_t)i * np + j;
                        const uint16_t hb = bf16_rn((float)x);
                        hih[o] = hb;
                        loh[o] = bf16_rn((float)(x - (double)bf16_to_f(hb)));
                        ybh[b] = std::max(ybh[b], std::fabs(x));
                        R += std::fabs(J[b][(size_t)i * n + j]);
                    }
                    const double e = (std::ldexp(1.0, -15) * 4.0 * 0.25 + 2.1 * n * std::ldexp(1.0, -24)) * R +
                                     std::ldexp(1.0, -23) * (std::fabs(h[b][i]) + R);
                    emax = std::max(emax, e);
                    // |a_i| = 2 |F_i| and |F_i| <= |h_i| + sum_j |J_ij| in every state
                    abh[b] = std::max(abh[b], 2.0 * (std::fabs(h[b][i]) + R));
                }
                ebfh[b] = emax;
            }
            if (h16) {
                // fl16(4J), nearest even; every |a| and |4J| must stay far inside the FP16 range
                std::vector<uint16_t> j16((size_t)jtot, 0);
                for (int b = 0; b < n_inst; ++b) {
                    if (abh[b] + ybh[b] > 16384.0) {
                        r2 = fail(ISING_ERR_INVALID_ARG, "instance %d: |a| can reach %g, too large for the FP16 scan",
                                  b, abh[b]);
                        break;
                    }
                    const int n = N[b], np = hd->Npad[b];
                    for (int i = 0; i < n; ++i)
                        for (int j = 0; j < n; ++j) {
                            const _Float16 v = (_Float16)(4.0 * J[b][(size_t)i * n + j]);
                            uint16_t u;
                            std::memcpy(&u, &v, 2);
                            j16[joff[b] + (size_t)i * np + j] = u;
                        }
                }
                cp(dJ16, j16.data(), sizeof(uint16_t) * j16.size());
            }
            cp(dJhi, hih.data(), sizeof(uint16_t) * hih.size());
            cp(dJlo, loh.data(), sizeof(uint16_t) * loh.size());
            cp(dyb, ybh.data(), sizeof(double) * n_inst);
            cp(debf, ebfh.data(), sizeof(double) * n_inst);
            cp(dab, abh.data(), sizeof(double) * n_inst);
        }
        std::vector<float> rmh;
        if (sb) {
            // site bound: max_j |4J_ij| per row, rounded up to FP32
            rmh.assign((size_t)n_inst * lay.Npmax, 0.f);
            for (int b = 0; b < n_inst; ++b) {
                const int n = N[b];
                for (int i = 0; i < n; ++i) {
                    double m = 0.0;
                    for (int j = 0; j < n; ++j) m = std::max(m, std::fabs(4.0 * J[b][(size_t)i * n + j]));
                    float f = (float)m;
                    if ((double)f < m) f = std::nextafter(f, INFINITY);
                    rmh[(size_t)b * lay.Npmax + i] = f;
                }
            }
            cp(drm, rmh.data(), sizeof(float) * rmh.size());
        }
        std::vector<double> fsch(n_inst, 1.0);
        for (int b = 0; b < n_inst; ++b) fsch[b] = fq_ok ? std::ldexp(1.0, -fgrid[b]) : 1.0;
        cp(dfsc, fsch.data(), sizeof(double) * n_inst);
        std::vector<uint16_t> jnh;
        if (cfg->form == ISING_FORM_LEARNED) {
            // bf16(sqrt(N) J_ij), rounded to nearest even, for the scoring network's features
            jnh.assign((size_t)jtot, 0);
            for (int b = 0; b < n_inst; ++b) {
                const int n = N[b], np = hd->Npad[b];
                const double sq = std::sqrt((double)n);
                for (int i = 0; i < n; ++i)
                    for (int j = 0; j < n; ++j) {
                        const float f = (float)(sq * J[b][(size_t)i * n + j]);
                        uint32_t u;
                        std::memcpy(&u, &f, 4);
                        u += 0x7FFFu + ((u >> 16) & 1u);
                        jnh[joff[b] + (size_t)i * np + j] = (uint16_t)(u >> 16);
                    }
            }
            cp(dJn, jnh.data(), sizeof(uint16_t) * jnh.size());
        }
        if (r2 == ISING_OK) {
            hipError_t e = hipMemsetAsync(lay.ctr, 0, 16 * sizeof(unsigned long long), sm);
            if (e == hipSuccess) e = hipMemsetAsync(lay.flags, 0, 8 * sizeof(int), sm);
            if (e == hipSuccess && hd->timing) e = hipEventRecord(hd->ev[0], sm);
            if (e == hipSuccess) e = launch_init_fields(lay, dx0, sm);
            if (e == hipSuccess && lay.form == ISING_FORM_SPLIT_BF16) {
                e = hipMemsetAsync(hd->d_maxerr, 0, sizeof(double), sm);
                if (e == hipSuccess) e = launch_init_split(lay, dx0, hd->d_maxerr, sm);
                if (e == hipSuccess) e = hipMemcpyAsync(&hd->split_err, hd->d_maxerr, sizeof(double),
                                                        hipMemcpyDeviceToHost, sm);
            }
            if (e == hipSuccess && hd->timing) e = hipEventRecord(hd->ev[1], sm);
            if (e == hipSuccess) e = hipStreamSynchronize(sm);
            if (e == hipSuccess && hd->timing) hd->t_init += elapsed_ms(hd->ev[0], hd->ev[1]);
            if (e != hipSuccess) r2 = fail(ISING_ERR_HIP, "initialisation kernels failed: %s", hipGetErrorString(e));
        }
        if (r2 != ISING_OK) return bail(r2);
    }
    int cus = 256;
    hipDeviceProp_t prop;
    std::memset(&prop, 0, sizeof prop);
    if (hipGetDeviceProperties(&prop, hd->device) == hipSuccess && prop.multiProcessorCount > 0)
        cus = prop.multiProcessorCount;
    prop.gcnArchName[sizeof(prop.gcnArchName) - 1] = 0;
    hd->scan_grid = cus * 16;
    hd->lay.scan_waves = hd->scan_grid;
    if (frontier_set_lds(lay) != hipSuccess) {
        (void)hipGetLastError();
        return bail(fail(ISING_ERR_HIP, "the frontier kernel cannot use its LDS"));
    }
    if (cfg->form == ISING_FORM_LEARNED) {
        const size_t lds = learn_lds_bytes(lay);
        if (learn_set_lds(lds) != hipSuccess) {
            (void)hipGetLastError();
            return bail(fail(ISING_ERR_HIP, "the ranking kernel cannot use %zu bytes of LDS", lds));
        }
        hd->learn_grid = cus * (lds + 2048 <= 80 * 1024 ? 2 : 1);
        uint64_t* tmp = nullptr;
        if (dalloc(hd, &tmp, (size_t)hd->learn_grid * lay.kmax) != ISING_OK) return bail(ISING_ERR_OUT_OF_MEMORY);
        lay.lr_tmp = tmp;
    }
    if (!weights.empty()) {
        if (hipMemcpyAsync(hd->d_mlp, weights.data(), sizeof(float) * MLP_NPARAM, hipMemcpyHostToDevice,
                           hd->stream) != hipSuccess || hipStreamSynchronize(hd->stream) != hipSuccess) {
            (void)hipGetLastError();
            return bail(fail(ISING_ERR_HIP, "copy of the network parameters failed"));
        }
        hd->lay.scorer = ISING_SCORER_NETWORK;
        hd->scorer_set = true;
    }
    if (cfg->tile_cache) hd->tile_cache = cfg->tile_cache;
    hd->cfg.tile_cache = nullptr;   // the caller's strings are not kept
    hd->cfg.mlp_weights = nullptr;
    hd->arch = prop.gcnArchName;
    {
        std::lock_guard<std::mutex> g(g_live_mu);
        g_live.insert(hd);
    }
    *out = hd;
    return ISING_OK;
}

// One pass of the step kernels; with timing on, events bracket each family.
static hipError_t launch_pass(ising_search* h, bool retry_mode)
{
    const Layout& lay = h->lay;
    hipStream_t st = h->stream;
    hipEvent_t* ev = h->ev;
    const bool tm = h->timing;
    hipError_t e = hipSuccess;
    auto rec = [&](int k) {
        if (tm && e == hipSuccess) e = hipEventRecord(ev[k], st);
    };
    rec(0);
    if (e == hipSuccess) e = launch_step_begin(lay, retry_mode, st);
    if (e == hipSuccess && !retry_mode) e = launch_frontier_plan(lay, st);
    rec(1);
    if (e == hipSuccess) e = launch_prep(lay, st, true, tm && lay.sb ? ev[7] : nullptr);
    rec(2);
    if (e == hipSuccess) e = launch_scan(lay, h->scan_grid, st);
    if (lay.form == ISING_FORM_LEARNED) {
        rec(6);
        if (e == hipSuccess) e = launch_learn(lay, h->learn_grid, st);
    }
    rec(3);
    if (e == hipSuccess) e = launch_merge(lay, st);
    if (e == hipSuccess) e = launch_fupdate(lay, st);
    if (e == hipSuccess && h->tracing && !retry_mode) e = launch_trace(lay, st);
    rec(4);
    if (e == hipSuccess) ++h->scan_launches;
    return e;
}

static void collect_times(ising_search* h)
{
    if (!h->timing) return;
    h->t_frontier += elapsed_ms(h->ev[0], h->ev[1]);
    h->t_prep += elapsed_ms(h->ev[1], h->ev[2]);
    if (h->lay.sb) h->t_bound += elapsed_ms(h->ev[1], h->ev[7]);
    if (h->lay.form == ISING_FORM_LEARNED) {
        h->t_scan += elapsed_ms(h->ev[2], h->ev[6]);
        h->t_learn += elapsed_ms(h->ev[6], h->ev[3]);
    } else {
        h->t_scan += elapsed_ms(h->ev[2], h->ev[3]);
    }
    h->t_merge += elapsed_ms(h->ev[3], h->ev[4]);
}

// Persistent mode: the kernels of one normal pass are captured once into a
// graph; each step replays it (retry passes after an overflow stay eager).
static hipError_t launch_graph_pass(ising_search* h)
{
    hipError_t e = hipSuccess;
    if (!h->gexec) {
        const bool tm = h->timing;
        h->timing = false;   // no events inside the captured pass
        e = hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t e2 = launch_pass(h, false);
            --h->scan_launches;
            e = hipStreamEndCapture(h->stream, &h->graph);
            if (e == hipSuccess) e = e2;
        }
        h->timing = tm;
        if (e == hipSuccess) e = hipGraphInstantiate(&h->gexec, h->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) return e;
    }
    if (h->timing) e = hipEventRecord(h->ev[0], h->stream);
    if (e == hipSuccess) e = hipGraphLaunch(h->gexec, h->stream);
    if (e == hipSuccess && h->timing) e = hipEventRecord(h->ev[5], h->stream);
    if (e == hipSuccess) ++h->scan_launches;
    return e;
}

// Doubles every search's candidate buffer, up to MAX_SURV_CAP records.  The
// stream is idle (sync_flags waited for it), so the old buffer can go.  The
// captured steps hold the old layout and are dropped.
static int grow_surv(ising_search* h)
{
    Layout& lay = h->lay;
    if (lay.cap_surv >= MAX_SURV_CAP)
        return fail(ISING_ERR_CAPACITY,
                    "a search has more candidates at its cut than %d records hold, and the buffer cannot grow",
                    lay.cap_surv);
    const int cap = lay.cap_surv > MAX_SURV_CAP / 2 ? MAX_SURV_CAP : 2 * lay.cap_surv;
    Surv* grown = nullptr;
    int rc = dalloc(h, &grown, (size_t)lay.S * cap);
    if (rc != ISING_OK) return rc;
    for (size_t k = 0; k < h->allocs.size(); ++k) {
        if (h->allocs[k] == static_cast<void*>(lay.surv)) {
            (void)hipFree(h->allocs[k]);
            h->allocs.erase(h->allocs.begin() + (long)k);
            break;
        }
    }
    lay.surv = grown;
    lay.cap_surv = cap;
    drop_graph(h);
    return ISING_OK;
}

// After a pass whose flags are on the host: re-scan the searches whose
// candidate buffer filled, with the cut their stored candidates give, until
// every one has committed.  A cut that cannot move (the stored records are
// copies of fewer than M distinct states) doubles the buffer first.
static int finish_retries(ising_search* h, bool collect)
{
    int guard = 0;
    while (h->flags_h[FLAG_OVERFLOW] > 0) {
        if (h->flags_h[FLAG_STUCK] > 0 || ++guard > 64) {
            int rc = grow_surv(h);
            if (rc != ISING_OK) return rc;
            guard = 0;
        }
        hipError_t e = launch_pass(h, true);
        if (e != hipSuccess) {
            h->broken = true;
            return fail(ISING_ERR_HIP, "retry launch failed: %s", hipGetErrorString(e));
        }
        int rc = sync_flags(h);
        if (rc != ISING_OK) {
            h->broken = true;
            return rc;
        }
        if (collect) collect_times(h);
    }
    return ISING_OK;
}

static int do_step(ising_search* h, int32_t* n_active)
{
    const Layout& lay = h->lay;
    if (lay.form == ISING_FORM_LEARNED && !h->scorer_set)
        return fail(ISING_ERR_BAD_STATE, "the learned form needs ising_search_set_scorer before stepping");
    hipError_t e = h->persistent ? launch_graph_pass(h) : launch_pass(h, false);
    if (e != hipSuccess) {
        h->broken = true;
        return fail(ISING_ERR_HIP, "step launch failed: %s", hipGetErrorString(e));
    }
    int rc = sync_flags(h);
    if (rc != ISING_OK) {
        h->broken = true;
        return rc;
    }
    if (h->persistent) {
        if (h->timing) h->t_step += elapsed_ms(h->ev[0], h->ev[5]);
    } else {
        collect_times(h);
    }
    rc = finish_retries(h, true);
    if (rc != ISING_OK) return rc;
    h->final_dirty = true;
    if (n_active) *n_active = h->flags_h[FLAG_ACTIVE];
    return ISING_OK;
}

// Up to graph_steps steps as one replayed graph.  A step that finds every
// search stable, or a full candidate buffer, halts the later steps on the
// device (they return at once); the full buffer's step then finishes with
// retry passes here.  *done receives the steps taken, *n_active the active
// searches after the last of them.
static int do_graph_steps(ising_search* h, int32_t* done, int32_t* n_active)
{
    const Layout& lay = h->lay;
    const int k = h->graph_steps;
    hipError_t e = hipSuccess;
    if (!h->gexec_k) {
        const bool tm = h->timing;
        h->timing = false;   // no events inside the captured steps
        e = hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t e2 = launch_graph_begin(lay, h->stream);
            for (int t = 0; t < k && e2 == hipSuccess; ++t) {
                e2 = launch_pass(h, false);
                --h->scan_launches;
                if (e2 == hipSuccess) e2 = launch_step_end(lay, t, h->stream);
            }
            e = hipStreamEndCapture(h->stream, &h->graph_k);
            if (e == hipSuccess) e = e2;
        }
        h->timing = tm;
        if (e == hipSuccess) e = hipGraphInstantiate(&h->gexec_k, h->graph_k, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            h->broken = true;
            return fail(ISING_ERR_HIP, "capture of %d steps failed: %s", k, hipGetErrorString(e));
        }
    }
    if (h->timing) e = hipEventRecord(h->ev[0], h->stream);
    if (e == hipSuccess) e = hipGraphLaunch(h->gexec_k, h->stream);
    if (e == hipSuccess && h->timing) e = hipEventRecord(h->ev[5], h->stream);
    int sa[MAX_GRAPH_STEPS];
    if (e == hipSuccess) e = hipMemcpyAsync(sa, lay.step_active, sizeof(int) * k, hipMemcpyDeviceToHost, h->stream);
    if (e != hipSuccess) {
        h->broken = true;
        return fail(ISING_ERR_HIP, "graph launch failed: %s", hipGetErrorString(e));
    }
    int rc = sync_flags(h);
    if (rc != ISING_OK) {
        h->broken = true;
        return rc;
    }
    if (h->timing) h->t_step += elapsed_ms(h->ev[0], h->ev[5]);
    const bool halted = h->flags_h[FLAG_HALT] != 0;
    const int steps = halted ? h->flags_h[FLAG_HALT_STEP] + 1 : k;
    h->scan_launches += steps;
    int active = sa[steps - 1];
    if (halted) {
        // clear the halt so that eager passes run
        e = launch_graph_begin(lay, h->stream);
        if (e != hipSuccess) {
            h->broken = true;
            return fail(ISING_ERR_HIP, "halt clear failed: %s", hipGetErrorString(e));
        }
        if (h->flags_h[FLAG_OVERFLOW] > 0) {
            rc = finish_retries(h, true);
            if (rc != ISING_OK) return rc;
            active = h->flags_h[FLAG_ACTIVE];
        }
    }
    h->final_dirty = true;
    *done = steps;
    *n_active = active;
    return ISING_OK;
}

// One step that first chooses the states per scan item for every distinct N:
// after the frontier and the per-state preparation, the scan (which only
// appends survivors, so it can be repeated after clearing them) is timed for
// each candidate, one N bucket at a time with the others held at their best.
extern "C" int ising_search_autotune(ising_search_t* s, int32_t* n_active)
{
    g_err.clear();
    int rc = check_handle(s);
    if (rc != ISING_OK) return rc;
    if (s->lay.form == ISING_FORM_LEARNED && !s->scorer_set)
        return fail(ISING_ERR_BAD_STATE, "the learned form needs ising_search_set_scorer before stepping");
    // tuned tiles are timed against the per-step choice; the captured step
    // holds the choice by value
    if (s->lay.sc_auto) {
        s->lay.sc_auto = 0;
        drop_graph(s);
    }
    const Layout& lay = s->lay;
    hipStream_t st = s->stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return fail(ISING_ERR_HIP, "hipEventCreate failed");
    }
    static const int cand[] = {16, 32, 64, 128, 256};
    std::vector<int> sizes(s->N);
    std::sort(sizes.begin(), sizes.end());
    sizes.erase(std::unique(sizes.begin(), sizes.end()), sizes.end());
    hipError_t e = launch_step_begin(lay, false, st);
    if (e == hipSuccess) e = launch_frontier_plan(lay, st);
    auto scan_ms = [&](float& ms, bool count) -> hipError_t {
        hipError_t r = hipMemcpyAsync(s->d_scb, s->sc_h.data(), sizeof(int) * lay.B, hipMemcpyHostToDevice, st);
        if (r == hipSuccess) r = launch_plan_only(lay, st);
        if (r == hipSuccess) r = launch_clear_survivors(lay, st);
        if (r == hipSuccess) r = launch_prep(lay, st, count);
        if (r == hipSuccess) r = hipEventRecord(e0, st);
        if (r == hipSuccess) r = launch_scan(lay, s->scan_grid, st);
        if (r == hipSuccess) r = hipEventRecord(e1, st);
        if (r == hipSuccess) r = hipStreamSynchronize(st);
        if (r == hipSuccess) ms = elapsed_ms(e0, e1);
        return r;
    };
    // sizes the cache lists take its tiles untimed
    const bool cache = !s->tile_cache.empty();
    std::vector<char> cached(sizes.size(), 0);
    int cached_per_step = 1;
    for (size_t k = 0; cache && k < sizes.size(); ++k) {
        int v = 0, a = 0;
        read_tile_cache(s->tile_cache, TileKey{s->arch, lay.form, s->cfg.flags, sizes[k], lay.M}, v, a);
        if (v > 0) {
            cached[k] = 1;
            cached_per_step &= a;
            for (int b = 0; b < lay.B; ++b)
                if (s->N[b] == sizes[k]) s->sc_h[b] = v;
        }
    }
    const bool all_cached = cache && std::all_of(cached.begin(), cached.end(), [](char c) { return c != 0; });
    for (size_t k = 0; k < sizes.size() && e == hipSuccess; ++k) {
        if (cached[k]) continue;
        int best = -1;
        float best_ms = 0.f;
        for (int c : cand) {
            for (int b = 0; b < lay.B; ++b)
                if (s->N[b] == sizes[k]) s->sc_h[b] = c;
            float ms = 0.f;
            e = scan_ms(ms, false);
            if (e != hipSuccess) break;
            if (best < 0 || ms < best_ms) {
                best = c;
                best_ms = ms;
            }
        }
        for (int b = 0; b < lay.B; ++b)
            if (s->N[b] == sizes[k]) s->sc_h[b] = best;
    }
    // the per-step choice competes with the tuned tiles on this step's frontier
    if (e == hipSuccess && s->sc_auto_ok && all_cached) {
        s->lay.sc_auto = cached_per_step;
    } else if (e == hipSuccess && s->sc_auto_ok) {
        float ms_t = 0.f, ms_a = 0.f;
        e = scan_ms(ms_t, false);
        if (e == hipSuccess) {
            s->lay.sc_auto = 1;
            e = scan_ms(ms_a, false);
        }
        if (e == hipSuccess && !(ms_a < ms_t)) s->lay.sc_auto = 0;
    }
    // the sizes tuned here go to the cache
    for (size_t k = 0; cache && k < sizes.size() && e == hipSuccess; ++k) {
        if (cached[k]) continue;
        int v = 0;
        for (int b = 0; b < lay.B; ++b)
            if (s->N[b] == sizes[k]) v = s->sc_h[b];
        rc = append_tile_cache(s->tile_cache, TileKey{s->arch, lay.form, s->cfg.flags, sizes[k], lay.M}, v,
                               s->lay.sc_auto);
        if (rc != ISING_OK) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            return rc;
        }
    }
    // the step itself with the chosen tiles
    float ms = 0.f;
    if (e == hipSuccess) e = scan_ms(ms, true);
    if (e == hipSuccess && lay.form == ISING_FORM_LEARNED) e = launch_learn(lay, s->learn_grid, st);
    if (e == hipSuccess) e = launch_merge(lay, st);
    if (e == hipSuccess) e = launch_fupdate(lay, st);
    if (e == hipSuccess && s->tracing) e = launch_trace(lay, st);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) {
        s->broken = true;
        return fail(ISING_ERR_HIP, "autotune step failed: %s", hipGetErrorString(e));
    }
    ++s->scan_launches;
    rc = sync_flags(s);
    if (rc != ISING_OK) {
        s->broken = true;
        return rc;
    }
    rc = finish_retries(s, false);
    if (rc != ISING_OK) return rc;
    s->final_dirty = true;
    if (n_active) *n_active = s->flags_h[FLAG_ACTIVE];
    return ISING_OK;
}

extern "C" int ising_search_get_tuning(ising_search_t* s, int32_t* states_per_item)
{
    g_err.clear();
    int rc = check_handle(s);
    if (rc != ISING_OK) return rc;
    if (!states_per_item) return fail(ISING_ERR_INVALID_ARG, "NULL output pointer");
    if (s->lay.sc_auto) {
        // chosen by the last step's plan
        HIP_TRY(hipMemcpyAsync(states_per_item, s->d_scb, sizeof(int32_t) * s->lay.B, hipMemcpyDeviceToHost,
                               s->stream));
        HIP_TRY(hipStreamSynchronize(s->stream));
        return ISING_OK;
    }
    for (int b = 0; b < s->lay.B; ++b) states_per_item[b] = s->sc_h[b];
    return ISING_OK;
}

// clear the device maximum of |F~ - F| with a kernel (kept out of hipMemset so a
// caller may capture the reset into a graph)
__global__ void k_clear_double(double* p) { *p = 0.0; }

static hipError_t launch_clear_err(ising_search* s)
{
    hipLaunchKernelGGL(k_clear_double, dim3(1), dim3(1), 0, s->stream, s->d_maxerr);
    return hipGetLastError();
}

extern "C" int ising_search_reset(ising_search_t* s)
{
    g_err.clear();
    int rc = check_handle(s);
    if (rc != ISING_OK) return rc;
    hipError_t e = hipSuccess;
    if (s->timing) e = hipEventRecord(s->ev[0], s->stream);
    if (e == hipSuccess) e = launch_init_fields(s->lay, s->x0, s->stream);
    if (e == hipSuccess && s->lay.form == ISING_FORM_SPLIT_BF16) {
        e = launch_clear_err(s);
        if (e == hipSuccess) e = launch_init_split(s->lay, s->x0, s->d_maxerr, s->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(&s->split_err, s->d_maxerr, sizeof(double), hipMemcpyDeviceToHost, s->stream);
    }
    if (e == hipSuccess && s->timing) e = hipEventRecord(s->ev[1], s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) {
        s->broken = true;
        return fail(ISING_ERR_HIP, "reset kernels failed: %s", hipGetErrorString(e));
    }
    if (s->timing) s->t_init += elapsed_ms(s->ev[0], s->ev[1]);
    s->final_dirty = true;
    return ISING_OK;
}

extern "C" int ising_search_step(ising_search_t* s, int32_t* n_active)
{
    g_err.clear();
    int rc = check_handle(s);
    if (rc != ISING_OK) return rc;
    return do_step(s, n_active);
}

extern "C" int ising_search_run(ising_search_t* s, int32_t max_iters, int32_t* iters_done)
{
    g_err.clear();
    int rc = check_handle(s);
    if (rc != ISING_OK) return rc;
    const int cap = max_iters > 0 ? max_iters : s->cfg.max_iters;
    int it = 0;
    int active = 1;
    if (s->lay.form == ISING_FORM_LEARNED && !s->scorer_set)
        return fail(ISING_ERR_BAD_STATE, "the learned form needs ising_search_set_scorer before stepping");
    while (it < cap && active > 0) {
        // persistent mode: graph_steps steps per replayed graph while the cap allows
        if (s->persistent && s->graph_steps > 1 && cap - it >= s->graph_steps) {
            int done = 0;
            rc = do_graph_steps(s, &done, &active);
            it += done;
        } else {
            rc = do_step(s, &active);
            ++it;
        }
        if (rc != ISING_OK) {
            if (iters_done) *iters_done = it;
            return rc;
        }
    }
    if (iters_done) *iters_done = it;
    return active > 0 ? ISING_NOT_CONVERGED : ISING_OK;
}

extern "C" int ising_search_get_states(ising_search_t* s, int32_t instance, uint64_t* bits_out, double* E_out,
                                       int32_t* count)
{
    g_err.clear();
    int rc = check_handle(s);
    if (rc != ISING_OK) return rc;
    if (instance < 0 || instance >= s->lay.B)
        return fail(ISING_ERR_INVALID_ARG, "instance %d outside [0, %d)", instance, s->lay.B);
    if (!bits_out || !E_out || !count) return fail(ISING_ERR_INVALID_ARG, "NULL output pointer");
    const Layout& lay = s->lay;
    if (s->final_dirty) {
        hipError_t e = launch_final(lay, s->stream);
        if (e != hipSuccess) {
            s->broken = true;
            return fail(ISING_ERR_HIP, "merge launch failed: %s", hipGetErrorString(e));
        }
        s->final_dirty = false;
    }
    int n = 0;
    const int W = words_of(s->N[instance]);
    std::vector<uint64_t> tmp((size_t)lay.M * lay.Wmax);
    HIP_TRY(hipMemcpyAsync(&n, lay.out_count + instance, sizeof(int), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipMemcpyAsync(tmp.data(), lay.out_bits + (size_t)instance * lay.M * lay.Wmax,
                           tmp.size() * sizeof(uint64_t), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipMemcpyAsync(E_out, lay.out_E + (size_t)instance * lay.M, sizeof(double) * lay.M,
                           hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    for (int k = 0; k < n; ++k)
        for (int w = 0; w < W; ++w) bits_out[(size_t)k * W + w] = tmp[(size_t)k * lay.Wmax + w];
    *count = n;
    return ISING_OK;
}

extern "C" int ising_search_get_search(ising_search_t* s, int32_t search, uint64_t* bits_out, double* E_out,
                                       uint8_t* front_out, int32_t* count)
{
    g_err.clear();
    int rc = check_handle(s);
    if (rc != ISING_OK) return rc;
    const Layout& lay = s->lay;
    if (search < 0 || search >= lay.S) return fail(ISING_ERR_INVALID_ARG, "search %d outside [0, %d)", search, lay.S);
    if (!bits_out || !E_out || !count) return fail(ISING_ERR_INVALID_ARG, "NULL output pointer");
    const int M = lay.M;
    const size_t M2 = 2 * (size_t)M;
    int nk = 0;
    std::vector<int> kept(M);
    std::vector<uint64_t> bits(M2 * lay.Wmax);
    std::vector<double> E(M2);
    std::vector<uint8_t> fr(M2);
    HIP_TRY(hipMemcpyAsync(&nk, lay.nkept + search, sizeof(int), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipMemcpyAsync(kept.data(), lay.kept + (size_t)search * M, sizeof(int) * M, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipMemcpyAsync(bits.data(), lay.bits + (size_t)search * M2 * lay.Wmax, sizeof(uint64_t) * bits.size(),
                           hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipMemcpyAsync(E.data(), lay.E + (size_t)search * M2, sizeof(double) * M2, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipMemcpyAsync(fr.data(), lay.fresh + (size_t)search * M2, M2, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    const int W = words_of(s->N[search / lay.L]);
    for (int k = 0; k < nk; ++k) {
        const int slot = kept[k];
        for (int w = 0; w < W; ++w) bits_out[(size_t)k * W + w] = bits[(size_t)slot * lay.Wmax + w];
        E_out[k] = E[slot];
        if (front_out) front_out[k] = fr[slot];
    }
    *count = nk;
    return ISING_OK;
}

extern "C" int ising_search_set_search(ising_search_t* s, int32_t search, const uint64_t* bits,
                                       const uint8_t* front, int32_t count)
{
    g_err.clear();
    int rc = check_handle(s);
    if (rc != ISING_OK) return rc;
    const Layout& lay = s->lay;
    if (search < 0 || search >= lay.S) return fail(ISING_ERR_INVALID_ARG, "search %d outside [0, %d)", search, lay.S);
    if (count < 1 || count > lay.M) return fail(ISING_ERR_INVALID_ARG, "count %d outside [1, M]", count);
    if (!bits) return fail(ISING_ERR_INVALID_ARG, "bits is NULL");
    const int n = s->N[search / lay.L];
    const int W = words_of(n);
    const int tail = n & 63;
    int sector = -1;
    if (lay.h1 == H1_EXCHANGE) {
        // the sector of the search: the number of down spins of its initial state
        std::vector<uint64_t> w0(lay.Wmax);
        HIP_TRY(hipMemcpyAsync(w0.data(), s->x0 + (size_t)search * lay.Wmax, sizeof(uint64_t) * lay.Wmax,
                               hipMemcpyDeviceToHost, s->stream));
        HIP_TRY(hipStreamSynchronize(s->stream));
        sector = 0;
        for (int w = 0; w < W; ++w) sector += __builtin_popcountll(w0[w]);
    }
    for (int k = 0; k < count; ++k) {
        if (tail && (bits[(size_t)k * W + W - 1] >> tail))
            return fail(ISING_ERR_INVALID_ARG, "state %d has bits at positions >= N", k);
        if (sector >= 0) {
            int downs = 0;
            for (int w = 0; w < W; ++w) downs += __builtin_popcountll(bits[(size_t)k * W + w]);
            if (downs != sector)
                return fail(ISING_ERR_INVALID_ARG, "state %d has %d down spins; the search's sector has %d", k, downs,
                            sector);
        }
        for (int q = 0; q < k; ++q)
            if (std::memcmp(bits + (size_t)k * W, bits + (size_t)q * W, W * sizeof(uint64_t)) == 0)
                return fail(ISING_ERR_INVALID_ARG, "states %d and %d are equal", q, k);
    }
    const int M = lay.M;
    const size_t M2 = 2 * (size_t)M;
    std::vector<uint64_t> hb((size_t)count * lay.Wmax, 0);
    for (int k = 0; k < count; ++k)
        for (int w = 0; w < W; ++w) hb[(size_t)k * lay.Wmax + w] = bits[(size_t)k * W + w];
    std::vector<uint8_t> hf(M2, 0);
    for (int k = 0; k < count; ++k) hf[k] = front ? (front[k] ? 1 : 0) : 1;
    HIP_TRY(hipMemcpyAsync(lay.bits + (size_t)search * M2 * lay.Wmax, hb.data(), hb.size() * sizeof(uint64_t),
                           hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipMemcpyAsync(lay.fresh + (size_t)search * M2, hf.data(), M2, hipMemcpyHostToDevice, s->stream));
    hipError_t e = launch_fields_for(lay, search, count, s->stream);
    if (e != hipSuccess) return fail(ISING_ERR_HIP, "field kernel failed: %s", hipGetErrorString(e));
    // order the kept list by (E, psi) on the host from the computed energies
    std::vector<double> E(count);
    HIP_TRY(hipMemcpyAsync(E.data(), lay.E + (size_t)search * M2, sizeof(double) * count, hipMemcpyDeviceToHost,
                           s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    std::vector<int> order(count);
    for (int k = 0; k < count; ++k) order[k] = k;
    auto less = [&](int a, int b) {
        if (E[a] != E[b]) return E[a] < E[b];
        for (int w = W - 1; w >= 0; --w) {
            const uint64_t x = bits[(size_t)a * W + w], y = bits[(size_t)b * W + w];
            if (x != y) return x < y;
        }
        return false;
    };
    for (int i = 1; i < count; ++i)
        for (int j = i; j > 0 && less(order[j], order[j - 1]); --j) std::swap(order[j], order[j - 1]);
    const int one = 1, zero = 0;
    HIP_TRY(hipMemcpyAsync(lay.kept + (size_t)search * M, order.data(), sizeof(int) * count, hipMemcpyHostToDevice,
                           s->stream));
    HIP_TRY(hipMemcpyAsync(lay.nkept + search, &count, sizeof(int), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipMemcpyAsync(lay.active + search, &one, sizeof(int), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipMemcpyAsync(lay.retry + search, &zero, sizeof(int), hipMemcpyHostToDevice, s->stream));
    if (lay.form == ISING_FORM_LEARNED) {
        // installed states have not had their pairs enumerated; the next step ranks
        HIP_TRY(hipMemsetAsync(lay.xfull + (size_t)search * M2, 0, M2, s->stream));
        HIP_TRY(hipMemcpyAsync(lay.mode + search, &zero, sizeof(int), hipMemcpyHostToDevice, s->stream));
    }
    HIP_TRY(hipStreamSynchronize(s->stream));
    s->final_dirty = true;
    return ISING_OK;
}

extern "C" int ising_search_get_stats(ising_search_t* s, ising_stats_t* out)
{
    g_err.clear();
    int rc = check_handle(s);
    if (rc != ISING_OK) return rc;
    if (!out) return fail(ISING_ERR_INVALID_ARG, "out is NULL");
    unsigned long long c[16];
    HIP_TRY(hipMemcpyAsync(c, s->lay.ctr, sizeof c, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    std::memset(out, 0, sizeof *out);
    out->steps = c[CTR_STEPS];
    out->pair_evals = c[CTR_PAIRS];
    out->single_evals = c[CTR_SINGLES];
    out->frontier_states = c[CTR_FRONTIER];
    out->survivors = c[CTR_SURV];
    out->retries = c[CTR_RETRY];
    out->fallbacks = c[CTR_FALLBACK];
    out->scan_launches = s->scan_launches;
    out->scan_ms = s->t_scan;
    out->merge_ms = s->t_merge;
    out->frontier_ms = s->t_frontier;
    out->prep_ms = s->t_prep;
    out->init_ms = s->t_init;
    out->step_ms = s->t_step;
    out->split_field_err = s->split_err;
    out->scored_pairs = c[CTR_SCORED];
    out->ranked_states = c[CTR_LEARNED];
    out->trace_samples = c[CTR_TRACE];
    out->learn_ms = s->t_learn;
    out->bounded_states = c[CTR_BOUNDED];
    out->surv_capacity = (uint64_t)s->lay.cap_surv;
    out->bound_ms = s->t_bound;
    out->field_bytes = s->lay.Fq ? 4 : 8;
    return ISING_OK;
}

extern "C" void ising_search_destroy(ising_search_t* s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> g(g_live_mu);
        if (!g_live.erase(s)) return;
    }
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    else (void)hipDeviceSynchronize();
    free_all(s);
    delete s;
}

// ------------------------------------------------------------------ learned-proposal form
extern "C" int ising_search_set_scorer(ising_search_t* s, int32_t scorer, const float* params, uint64_t seed)
{
    g_err.clear();
    int rc = check_handle(s);
    if (rc != ISING_OK) return rc;
    if (s->lay.form != ISING_FORM_LEARNED) return fail(ISING_ERR_INVALID_ARG, "the handle is not of the learned form");
    if (scorer < ISING_SCORER_NETWORK || scorer > ISING_SCORER_UNIFORM)
        return fail(ISING_ERR_INVALID_ARG, "scorer %d is not one of the scorers", scorer);
    if (scorer == ISING_SCORER_NETWORK) {
        if (!params) return fail(ISING_ERR_INVALID_ARG, "the network scorer needs its parameters");
        for (int k = 0; k < MLP_NPARAM; ++k)
            if (!std::isfinite(params[k])) return fail(ISING_ERR_INVALID_ARG, "parameter %d is not finite", k);
        HIP_TRY(hipMemcpyAsync(s->d_mlp, params, sizeof(float) * MLP_NPARAM, hipMemcpyHostToDevice, s->stream));
        HIP_TRY(hipStreamSynchronize(s->stream));
    }
    s->lay.scorer = scorer;
    s->lay.seed = seed;
    s->scorer_set = true;
    drop_graph(s);
    return ISING_OK;
}

extern "C" int ising_search_set_trace(ising_search_t* s, float* feat, uint8_t* label, int64_t capacity,
                                      int32_t pairs_per_state, float rate, uint64_t seed)
{
    g_err.clear();
    int rc = check_handle(s);
    if (rc != ISING_OK) return rc;
    if (s->lay.sb && feat)
        return fail(ISING_ERR_BAD_STATE, "trace capture reads every expanded state's a row, which the site bound skips");
    Layout& lay = s->lay;
    if (!feat || !label || capacity <= 0) {
        if (feat || label || capacity != 0) return fail(ISING_ERR_INVALID_ARG, "trace buffers: all NULL / 0 to stop");
        lay.tr_feat = nullptr;
        lay.tr_label = nullptr;
        lay.tr_cap = 0;
        s->tracing = false;
        drop_graph(s);
        return ISING_OK;
    }
    if (pairs_per_state < 0 || pairs_per_state > 1 << 20)
        return fail(ISING_ERR_INVALID_ARG, "pairs_per_state=%d outside [0, 2^20]", pairs_per_state);
    if (!(rate >= 0.f && rate <= 1.f)) return fail(ISING_ERR_INVALID_ARG, "rate outside [0, 1]");
    lay.tr_feat = feat;
    lay.tr_label = label;
    lay.tr_cap = capacity;
    lay.tr_neg = pairs_per_state;
    lay.tr_rate = rate;
    lay.seed = seed;
    s->tracing = true;
    const unsigned long long zero = 0;
    HIP_TRY(hipMemcpyAsync(lay.ctr + CTR_TRACE, &zero, sizeof zero, hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    drop_graph(s);
    return ISING_OK;
}

extern "C" int ising_search_get_trace_count(ising_search_t* s, int64_t* count)
{
    g_err.clear();
    int rc = check_handle(s);
    if (rc != ISING_OK) return rc;
    if (!count) return fail(ISING_ERR_INVALID_ARG, "count is NULL");
    unsigned long long c = 0;
    HIP_TRY(hipMemcpyAsync(&c, s->lay.ctr + CTR_TRACE, sizeof c, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    *count = (int64_t)c;
    return ISING_OK;
}

extern "C" int ising_search_get_proposals(ising_search_t* s, int32_t search, uint64_t* parent_bits, uint32_t* pairs,
                                          int32_t* n_pairs, int32_t max_parents, int32_t* n_parents, int32_t* mode)
{
    g_err.clear();
    int rc = check_handle(s);
    if (rc != ISING_OK) return rc;
    const Layout& lay = s->lay;
    if (!s->record) return fail(ISING_ERR_BAD_STATE, "the handle does not record proposals (ISING_FLAG_RECORD_PROPOSALS)");
    if (search < 0 || search >= lay.S) return fail(ISING_ERR_INVALID_ARG, "search %d outside [0, %d)", search, lay.S);
    if (!n_parents || !mode || (max_parents > 0 && (!parent_bits || !pairs || !n_pairs)))
        return fail(ISING_ERR_INVALID_ARG, "NULL output pointer");
    const int b = search / lay.L;
    const int W = words_of(s->N[b]);
    int nl = 0, md = 0;
    HIP_TRY(hipMemcpyAsync(&nl, lay.lr_count + b, sizeof(int), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipMemcpyAsync(&md, lay.last_mode + search, sizeof(int), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    std::vector<int> codes(nl > 0 ? nl : 1);
    const size_t base = (size_t)b * lay.fmax + (size_t)(lay.fmax - nl);
    if (nl > 0)
        HIP_TRY(hipMemcpyAsync(codes.data(), lay.fr_list + base, sizeof(int) * nl, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    int np = 0;
    std::vector<uint64_t> w(lay.Wmax);
    for (int k = 0; k < nl; ++k) {
        if (codes[k] / (2 * lay.M) != search) continue;
        if (np >= max_parents) return fail(ISING_ERR_CAPACITY, "more than max_parents=%d ranked parents", max_parents);
        const size_t fe = base + k;
        int cnt = 0;
        HIP_TRY(hipMemcpyAsync(&cnt, lay.prop_n + fe, sizeof(int), hipMemcpyDeviceToHost, s->stream));
        HIP_TRY(hipMemcpyAsync(w.data(), lay.fbits + fe * lay.Wmax, sizeof(uint64_t) * lay.Wmax,
                               hipMemcpyDeviceToHost, s->stream));
        HIP_TRY(hipStreamSynchronize(s->stream));
        if (cnt < 0 || cnt > lay.kmax) return fail(ISING_ERR_BAD_STATE, "corrupt proposal count %d", cnt);
        if (cnt > 0)
            HIP_TRY(hipMemcpyAsync(pairs + (size_t)np * lay.kmax, lay.prop + fe * lay.kmax, sizeof(uint32_t) * cnt,
                                   hipMemcpyDeviceToHost, s->stream));
        for (int q = 0; q < W; ++q) parent_bits[(size_t)np * W + q] = w[q];
        n_pairs[np] = cnt;
        ++np;
    }
    HIP_TRY(hipStreamSynchronize(s->stream));
    *n_parents = np;
    *mode = md;
    return ISING_OK;
}

extern "C" int32_t ising_search_topk(ising_search_t* s)
{
    if (check_handle(s) != ISING_OK) return -1;
    return s->lay.kmax;
}

// ------------------------------------------------------------------ training of the scoring network
namespace {
constexpr int64_t MLP_WS_GRID = 1024;   // blocks of the gradient kernel at most
int64_t mlp_ws_need() { return (MLP_WS_GRID * (MLP_NPARAM + 1) + MLP_NPARAM + 1) * (int64_t)sizeof(float); }
int have_device()
{
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        return fail(ISING_ERR_NO_DEVICE, "no HIP device available");
    }
    return ISING_OK;
}
}  // namespace

extern "C" int64_t ising_mlp_workspace_bytes(void) { return mlp_ws_need(); }

extern "C" int32_t ising_mlp_num_params(void) { return MLP_NPARAM; }

extern "C" int ising_mlp_forward(const float* params, const float* feat, int64_t n, float* logits, void* stream)
{
    g_err.clear();
    if (!params || !feat || !logits || n < 0) return fail(ISING_ERR_INVALID_ARG, "NULL pointer or n < 0");
    int rc = have_device();
    if (rc != ISING_OK) return rc;
    if (n == 0) return ISING_OK;
    hipError_t e = launch_mlp_forward(params, feat, n, logits, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail(ISING_ERR_HIP, "forward launch failed: %s", hipGetErrorString(e));
    return ISING_OK;
}

extern "C" int ising_mlp_loss_grad(const float* params, const float* feat, const uint8_t* label, int64_t n,
                                   float pos_weight, float* grad, float* loss, void* workspace, int64_t workspace_bytes,
                                   void* stream)
{
    g_err.clear();
    if (!params || !feat || !label || !grad || !workspace || n < 1)
        return fail(ISING_ERR_INVALID_ARG, "NULL pointer or n < 1");
    if (workspace_bytes < mlp_ws_need())
        return fail(ISING_ERR_INVALID_ARG, "workspace of %lld bytes < %lld", (long long)workspace_bytes,
                    (long long)mlp_ws_need());
    if (!(pos_weight > 0.f) || !std::isfinite(pos_weight)) return fail(ISING_ERR_INVALID_ARG, "pos_weight must be > 0");
    int rc = have_device();
    if (rc != ISING_OK) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    float* partial = static_cast<float*>(workspace);
    const int grid = mlp_grid_for(n);
    hipError_t e = launch_mlp_grad(params, feat, label, n, n, 0, -1, pos_weight, partial, grid, st);
    if (e == hipSuccess) e = launch_mlp_reduce(partial, grid, grad, loss, st);
    if (e != hipSuccess) return fail(ISING_ERR_HIP, "gradient launch failed: %s", hipGetErrorString(e));
    return ISING_OK;
}

// ------------------------------------------------------------------ gradient without allocation
// The partial gradients of at most MLP_NOALLOC_GRID blocks live in a
// file-scope device array (4,654,080 bytes), one copy per device, held until
// the process ends.  Host code never passes the array's name to a kernel: its
// device address is looked up once per device with hipGetSymbolAddress and
// kept in g_scratch_ptr.
namespace {
constexpr int MLP_NOALLOC_GRID = 256;
constexpr size_t MLP_NOALLOC_FLOATS = (size_t)MLP_NOALLOC_GRID * (MLP_NPARAM + 1);
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[MAX_DEVICES] = {};
}  // namespace

static __device__ __align__(256) float scratch[MLP_NOALLOC_FLOATS];

namespace {
int scratch_for_current_device(float** out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return fail(ISING_ERR_NO_DEVICE, "hipGetDevice failed");
    }
    if (dev < 0 || dev >= MAX_DEVICES) return fail(ISING_ERR_NO_DEVICE, "device %d outside [0, %d)", dev, MAX_DEVICES);
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(ISING_ERR_HIP, "hipGetSymbolAddress of the gradient scratch failed: %s", hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = static_cast<float*>(p);
    }
    *out = g_scratch_ptr[dev];
    return ISING_OK;
}
}  // namespace

extern "C" int ising_mlp_loss_grad_noalloc(const float* params, const float* feat, const uint8_t* label, int64_t n,
                                           float pos_weight, float* grad, float* loss, void* stream)
{
    g_err.clear();
    if (!params || !feat || !label || !grad || n < 1) return fail(ISING_ERR_INVALID_ARG, "NULL pointer or n < 1");
    if (!(pos_weight > 0.f) || !std::isfinite(pos_weight)) return fail(ISING_ERR_INVALID_ARG, "pos_weight must be > 0");
    int rc = have_device();
    if (rc != ISING_OK) return rc;
    float* partial = nullptr;
    rc = scratch_for_current_device(&partial);
    if (rc != ISING_OK) return rc;
    // at most MLP_NOALLOC_GRID blocks (rows of the scratch); more samples are
    // spread over them, so no sample count exceeds the scratch
    const int grid = std::min(mlp_grid_for(n), MLP_NOALLOC_GRID);
    hipStream_t st = static_cast<hipStream_t>(stream);
    // every block writes its whole row of partial sums, so the scratch needs no clearing
    hipError_t e = launch_mlp_grad(params, feat, label, n, n, 0, -1, pos_weight, partial, grid, st);
    if (e == hipSuccess) e = launch_mlp_reduce(partial, grid, grad, loss, st);
    if (e != hipSuccess) return fail(ISING_ERR_HIP, "gradient launch failed: %s", hipGetErrorString(e));
    return ISING_OK;
}

extern "C" int ising_mlp_adam(float* params, float* m, float* v, const float* grad, int32_t t, float lr, float beta1,
                              float beta2, float eps, void* stream)
{
    g_err.clear();
    if (!params || !m || !v || !grad) return fail(ISING_ERR_INVALID_ARG, "NULL pointer");
    if (t < 1 || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f) || !(lr > 0.f))
        return fail(ISING_ERR_INVALID_ARG, "Adam hyper-parameters out of range");
    int rc = have_device();
    if (rc != ISING_OK) return rc;
    const float c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, t)));
    const float c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, t)));
    hipError_t e = launch_mlp_adam(params, m, v, grad, lr, beta1, beta2, eps, c1, c2, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail(ISING_ERR_HIP, "Adam launch failed: %s", hipGetErrorString(e));
    return ISING_OK;
}

extern "C" int ising_mlp_train(float* params, float* m, float* v, const float* feat, const uint8_t* label, int64_t n,
                               int32_t batch, int32_t steps, int32_t t0, float lr, float pos_weight, uint64_t seed,
                               float* loss, void* workspace, int64_t workspace_bytes, void* stream)
{
    g_err.clear();
    if (!params || !m || !v || !feat || !label || !workspace || n < 1)
        return fail(ISING_ERR_INVALID_ARG, "NULL pointer or n < 1");
    if (batch < 1 || steps < 0 || t0 < 0) return fail(ISING_ERR_INVALID_ARG, "batch < 1, steps < 0 or t0 < 0");
    if (workspace_bytes < mlp_ws_need())
        return fail(ISING_ERR_INVALID_ARG, "workspace of %lld bytes < %lld", (long long)workspace_bytes,
                    (long long)mlp_ws_need());
    if (!(pos_weight > 0.f) || !std::isfinite(pos_weight) || !(lr > 0.f))
        return fail(ISING_ERR_INVALID_ARG, "pos_weight and lr must be > 0");
    int rc = have_device();
    if (rc != ISING_OK) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    float* partial = static_cast<float*>(workspace);
    float* grad = partial + MLP_WS_GRID * (MLP_NPARAM + 1);
    const int grid = mlp_grid_for(batch);
    const double b1 = 0.9, b2 = 0.999;
    for (int k = 0; k < steps; ++k) {
        const int t = t0 + k + 1;
        hipError_t e = launch_mlp_grad(params, feat, label, n, batch, seed, k + t0, pos_weight, partial, grid, st);
        if (e == hipSuccess) e = launch_mlp_reduce(partial, grid, grad, loss, st);
        if (e == hipSuccess)
            e = launch_mlp_adam(params, m, v, grad, lr, (float)b1, (float)b2, 1e-8f,
                                (float)(1.0 / (1.0 - std::pow(b1, t))), (float)(1.0 / (1.0 - std::pow(b2, t))), st);
        if (e != hipSuccess) return fail(ISING_ERR_HIP, "training launch failed: %s", hipGetErrorString(e));
    }
    return ISING_OK;
}

// ------------------------------------------------------------------ exhaustive enumeration
namespace {

// device buffers of one size group, freed on every exit path
struct BruteBufs {
    std::vector<void*> p;
    ~BruteBufs()
    {
        for (void* q : p) (void)hipFree(q);
    }
    template <class T>
    int get(T** out, size_t count)
    {
        void* v = nullptr;
        const size_t bytes = std::max<size_t>(count * sizeof(T), 8);
        if (hipMalloc(&v, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return fail(ISING_ERR_OUT_OF_MEMORY, "hipMalloc of %zu bytes failed", bytes);
        }
        p.push_back(v);
        *out = static_cast<T*>(v);
        return ISING_OK;
    }
};

}  // namespace

extern "C" int ising_brute_lowest(int32_t n_inst, const int32_t* N, const double* const* J, const double* const* h,
                                  int32_t K, uint64_t* bits_out, double* E_out, int32_t* count, void* stream)
{
    g_err.clear();
    if (n_inst < 1) return fail(ISING_ERR_INVALID_ARG, "n_inst=%d < 1", n_inst);
    if (!N || !J || !h || !bits_out || !E_out || !count) return fail(ISING_ERR_INVALID_ARG, "NULL array argument");
    if (K < 1 || K > BF_KMAX) return fail(ISING_ERR_INVALID_ARG, "K=%d outside [1, %d]", K, BF_KMAX);
    for (int b = 0; b < n_inst; ++b) {
        if (N[b] < 1 || N[b] > BF_NMAX) return fail(ISING_ERR_INVALID_ARG, "N[%d]=%d outside [1, %d]", b, N[b], BF_NMAX);
        if (!J[b] || !h[b]) return fail(ISING_ERR_INVALID_ARG, "NULL pointer for instance %d", b);
        const int n = N[b];
        double bound = 0.0;
        for (int i = 0; i < n; ++i) {
            if (!on_grid(h[b][i]))
                return fail(ISING_ERR_INVALID_ARG, "h[%d][%d]=%g is not a finite multiple of 2^-24", b, i, h[b][i]);
            bound += std::fabs(h[b][i]);
            if (J[b][(size_t)i * n + i] != 0.0)
                return fail(ISING_ERR_INVALID_ARG, "J[%d] has a nonzero diagonal at %d", b, i);
            for (int j = i + 1; j < n; ++j) {
                const double v = J[b][(size_t)i * n + j];
                if (!on_grid(v))
                    return fail(ISING_ERR_INVALID_ARG, "J[%d][%d,%d]=%g is not a finite multiple of 2^-24", b, i, j, v);
                if (v != J[b][(size_t)j * n + i])
                    return fail(ISING_ERR_INVALID_ARG, "J[%d] is not symmetric at (%d,%d)", b, i, j);
                bound += std::fabs(v);
            }
        }
        if (bound > 16777216.0)
            return fail(ISING_ERR_INVALID_ARG, "instance %d: sum |J_ij| + sum |h_i| = %g exceeds 2^24", b, bound);
    }
    int rc = have_device();
    if (rc != ISING_OK) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    static std::once_flag lds_once;
    static hipError_t lds_err = hipSuccess;
    std::call_once(lds_once, [] { lds_err = brute_sort_set_lds(); });
    if (lds_err != hipSuccess) return fail(ISING_ERR_HIP, "the sort kernel cannot use its LDS");

    std::vector<int> sizes(N, N + n_inst);
    std::sort(sizes.begin(), sizes.end());
    sizes.erase(std::unique(sizes.begin(), sizes.end()), sizes.end());
    for (int n : sizes) {
        std::vector<int> members;
        for (int b = 0; b < n_inst; ++b)
            if (N[b] == n) members.push_back(b);
        const int nb = (int)members.size();
        BruteBufs buf;
        double *dJ = nullptr, *dh = nullptr, *dD = nullptr, *dT = nullptr, *dE = nullptr;
        unsigned long long *dmin = nullptr, *dcnt = nullptr;
        BruteRec* drec = nullptr;
        int *dlist = nullptr, *dn = nullptr;
        uint64_t* dbits = nullptr;
        if ((rc = buf.get(&dJ, (size_t)nb * n * n)) || (rc = buf.get(&dh, (size_t)nb * n)) ||
            (rc = buf.get(&dD, (size_t)nb * BF_DSTRIDE)) || (rc = buf.get(&dT, nb)) || (rc = buf.get(&dmin, nb)) ||
            (rc = buf.get(&dcnt, nb)) || (rc = buf.get(&drec, (size_t)nb * BF_CAP)) || (rc = buf.get(&dlist, nb)) ||
            (rc = buf.get(&dn, nb)) || (rc = buf.get(&dbits, (size_t)nb * K)) || (rc = buf.get(&dE, (size_t)nb * K)))
            return rc;
        {
            std::vector<double> Jh((size_t)nb * n * n), hh((size_t)nb * n);
            std::vector<int> lst(nb);
            for (int k = 0; k < nb; ++k) {
                std::memcpy(Jh.data() + (size_t)k * n * n, J[members[k]], sizeof(double) * n * n);
                std::memcpy(hh.data() + (size_t)k * n, h[members[k]], sizeof(double) * n);
                lst[k] = k;
            }
            std::vector<unsigned long long> big(nb, ~0ull);
            HIP_TRY(hipMemcpyAsync(dJ, Jh.data(), sizeof(double) * Jh.size(), hipMemcpyHostToDevice, st));
            HIP_TRY(hipMemcpyAsync(dh, hh.data(), sizeof(double) * hh.size(), hipMemcpyHostToDevice, st));
            HIP_TRY(hipMemcpyAsync(dlist, lst.data(), sizeof(int) * nb, hipMemcpyHostToDevice, st));
            HIP_TRY(hipMemcpyAsync(dmin, big.data(), sizeof(unsigned long long) * nb, hipMemcpyHostToDevice, st));
            HIP_TRY(hipStreamSynchronize(st));   // the host vectors go out of scope
        }
        BruteArgs a{};
        a.N = n;
        a.n_list = nb;
        a.list = dlist;
        a.J = dJ;
        a.h = dh;
        a.D = dD;
        a.T = dT;
        a.emin = dmin;
        a.count = dcnt;
        a.rec = drec;
        hipError_t e = launch_brute_table(a, st);
        if (e == hipSuccess) e = launch_brute_pass(a, BF_MIN, st);
        if (e != hipSuccess) return fail(ISING_ERR_HIP, "enumeration launch failed: %s", hipGetErrorString(e));
        // the lowest energy of every instance, from its order-preserving image
        std::vector<unsigned long long> omin(nb);
        HIP_TRY(hipMemcpyAsync(omin.data(), dmin, sizeof(unsigned long long) * nb, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        std::vector<double> emin(nb);
        for (int k = 0; k < nb; ++k) {
            const unsigned long long o = omin[k];
            const unsigned long long u = (o >> 63) ? (o & 0x7FFFFFFFFFFFFFFFull) : ~o;
            std::memcpy(&emin[k], &u, 8);
        }
        // a threshold T_k per instance with want <= #{E <= T_k} <= BF_CAP: grow the
        // distance above the minimum fourfold until enough states lie below it,
        // then bisect while too many do
        const double total = std::ldexp(1.0, n);
        const long long want = (long long)std::min<double>(K, total);
        std::vector<double> T(nb, INFINITY);
        if (total > BF_CAP) {
            std::vector<double> lo(nb, -1.0), hi(nb, -1.0), d(nb);
            std::vector<int> open;
            for (int k = 0; k < nb; ++k) {
                double scale = 0.0;
                for (int i = 0; i < n; ++i) scale = std::max(scale, std::fabs(h[members[k]][i]));
                for (size_t q = 0; q < (size_t)n * n; ++q) scale = std::max(scale, std::fabs(J[members[k]][q]));
                d[k] = std::max(scale, 1.0) * std::ldexp(1.0, -6);
                open.push_back(k);
            }
            d.resize(nb);
            for (int it = 0; !open.empty(); ++it) {
                if (it > 400) return fail(ISING_ERR_HIP, "threshold search did not converge");
                for (int k = 0; k < nb; ++k) T[k] = -INFINITY;
                for (int k : open) T[k] = emin[k] + d[k];
                HIP_TRY(hipMemcpyAsync(dT, T.data(), sizeof(double) * nb, hipMemcpyHostToDevice, st));
                HIP_TRY(hipMemsetAsync(dcnt, 0, sizeof(unsigned long long) * nb, st));
                BruteArgs c = a;
                c.n_list = (int)open.size();
                HIP_TRY(hipMemcpyAsync(dlist, open.data(), sizeof(int) * open.size(), hipMemcpyHostToDevice, st));
                e = launch_brute_pass(c, BF_COUNT, st);
                if (e != hipSuccess) return fail(ISING_ERR_HIP, "count launch failed: %s", hipGetErrorString(e));
                std::vector<unsigned long long> cnt(nb);
                HIP_TRY(hipMemcpyAsync(cnt.data(), dcnt, sizeof(unsigned long long) * nb, hipMemcpyDeviceToHost, st));
                HIP_TRY(hipStreamSynchronize(st));
                std::vector<int> still;
                for (int k : open) {
                    const long long c2 = (long long)cnt[k];
                    if (c2 >= want && c2 <= BF_CAP) {
                        lo[k] = d[k];   // final
                        continue;
                    }
                    if (c2 < want) lo[k] = d[k];
                    else hi[k] = d[k];
                    if (hi[k] < 0) {
                        d[k] *= 4.0;
                    } else {
                        const double lo_k = std::max(lo[k], 0.0);
                        if (hi[k] - lo_k <= std::ldexp(1.0, -23))
                            return fail(ISING_ERR_CAPACITY,
                                        "instance %d: more than %d states tie at its %lld-th lowest energy",
                                        members[k], BF_CAP, want);
                        d[k] = 0.5 * (lo_k + hi[k]);
                    }
                    still.push_back(k);
                }
                open.swap(still);
            }
            for (int k = 0; k < nb; ++k) T[k] = emin[k] + lo[k];
        }
        std::vector<int> all(nb);
        for (int k = 0; k < nb; ++k) all[k] = k;
        HIP_TRY(hipMemcpyAsync(dlist, all.data(), sizeof(int) * nb, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(dT, T.data(), sizeof(double) * nb, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemsetAsync(dcnt, 0, sizeof(unsigned long long) * nb, st));
        e = launch_brute_pass(a, BF_COLLECT, st);
        if (e == hipSuccess) e = launch_brute_sort(a, K, dbits, dE, dn, st);
        if (e != hipSuccess) return fail(ISING_ERR_HIP, "collect launch failed: %s", hipGetErrorString(e));
        std::vector<unsigned long long> cnt(nb);
        std::vector<int> nout(nb);
        std::vector<uint64_t> ob((size_t)nb * K);
        std::vector<double> oE((size_t)nb * K);
        HIP_TRY(hipMemcpyAsync(cnt.data(), dcnt, sizeof(unsigned long long) * nb, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(nout.data(), dn, sizeof(int) * nb, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(ob.data(), dbits, sizeof(uint64_t) * ob.size(), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(oE.data(), dE, sizeof(double) * oE.size(), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        for (int k = 0; k < nb; ++k) {
            if (cnt[k] > (unsigned long long)BF_CAP || (long long)nout[k] < want)
                return fail(ISING_ERR_HIP, "instance %d: %llu states collected for %lld", members[k], cnt[k], want);
            const int b = members[k];
            std::memcpy(bits_out + (size_t)b * K, ob.data() + (size_t)k * K, sizeof(uint64_t) * nout[k]);
            std::memcpy(E_out + (size_t)b * K, oE.data() + (size_t)k * K, sizeof(double) * nout[k]);
            count[b] = nout[k];
        }
    }
    return ISING_OK;
}

// ------------------------------------------------------------------ best-first search (Alg. 2-4)
extern "C" int ising_bestfirst(int32_t n_inst, const int32_t* N, const double* const* J, const double* const* h,
                               int32_t L, const uint64_t* const* init_bits, int32_t K, int32_t I, int32_t flags,
                               uint64_t* merged_bits, double* merged_E, int32_t* merged_count,
                               uint64_t* search_bits, double* search_E, uint8_t* search_used, int32_t* search_born,
                               int32_t* search_count, int32_t* expanded, float* kernel_ms, void* stream)
{
    g_err.clear();
    if (n_inst < 1) return fail(ISING_ERR_INVALID_ARG, "n_inst=%d < 1", n_inst);
    if (L < 1) return fail(ISING_ERR_INVALID_ARG, "L=%d < 1", L);
    if ((long long)n_inst * L > (1 << 24)) return fail(ISING_ERR_INVALID_ARG, "too many searches");
    if (K < 0 || K + 1 > BFS_K1MAX) return fail(ISING_ERR_INVALID_ARG, "K=%d outside [0, %d]", K, BFS_K1MAX - 1);
    if (I < 0) return fail(ISING_ERR_INVALID_ARG, "I=%d < 0", I);
    if (flags & ~(ISING_FLAG_SINGLE_FLIPS | ISING_FLAG_EXCHANGE))
        return fail(ISING_ERR_INVALID_ARG, "flags 0x%x: only the H1 flags apply", flags);
    if ((flags & ISING_FLAG_SINGLE_FLIPS) && (flags & ISING_FLAG_EXCHANGE))
        return fail(ISING_ERR_INVALID_ARG, "single flips and exchanges are two different choices of H1");
    if (!N || !J || !h || !init_bits || !merged_bits || !merged_E || !merged_count)
        return fail(ISING_ERR_INVALID_ARG, "NULL array argument");
    const int h1 = (flags & ISING_FLAG_SINGLE_FLIPS) ? H1_SINGLES : ((flags & ISING_FLAG_EXCHANGE) ? H1_EXCHANGE : H1_FLIPS);
    int nmax = 0;
    for (int b = 0; b < n_inst; ++b) {
        if (N[b] < 1 || N[b] > BFS_NMAX)
            return fail(ISING_ERR_INVALID_ARG, "N[%d]=%d outside [1, %d]", b, N[b], BFS_NMAX);
        if (!J[b] || !h[b] || !init_bits[b]) return fail(ISING_ERR_INVALID_ARG, "NULL pointer for instance %d", b);
        nmax = std::max(nmax, (int)N[b]);
        const int n = N[b];
        double bound = 0.0;
        for (int i = 0; i < n; ++i) {
            if (!on_grid(h[b][i]))
                return fail(ISING_ERR_INVALID_ARG, "h[%d][%d]=%g is not a finite multiple of 2^-24", b, i, h[b][i]);
            bound += std::fabs(h[b][i]);
            if (J[b][(size_t)i * n + i] != 0.0)
                return fail(ISING_ERR_INVALID_ARG, "J[%d] has a nonzero diagonal at %d", b, i);
            for (int j = i + 1; j < n; ++j) {
                const double v = J[b][(size_t)i * n + j];
                if (!on_grid(v))
                    return fail(ISING_ERR_INVALID_ARG, "J[%d][%d,%d]=%g is not a finite multiple of 2^-24", b, i, j, v);
                if (v != J[b][(size_t)j * n + i])
                    return fail(ISING_ERR_INVALID_ARG, "J[%d] is not symmetric at (%d,%d)", b, i, j);
                bound += std::fabs(v);
            }
        }
        if (bound > 16777216.0)
            return fail(ISING_ERR_INVALID_ARG, "instance %d: sum |J_ij| + sum |h_i| = %g exceeds 2^24", b, bound);
        for (int l = 0; l < L; ++l)
            if (n < 64 && (init_bits[b][l] >> n))
                return fail(ISING_ERR_INVALID_ARG, "initial state %d of instance %d has bits at positions >= N", l, b);
    }
    const int K1 = K + 1;
    const int nchild = (h1 == H1_EXCHANGE ? 0 : nmax) + (h1 == H1_SINGLES ? 0 : nmax * (nmax - 1) / 2);
    int Cs = 1;
    while (Cs < nchild) Cs <<= 1;
    // the lists in LDS when they fit, else in global memory per block
    const BestFirstPlan plan = bestfirst_plan(K1, Cs);
    int rc = have_device();
    if (rc != ISING_OK) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = bestfirst_set_lds(plan);
    if (e != hipSuccess)
        return fail(ISING_ERR_HIP, "the best-first kernels cannot use %zu and %zu bytes of LDS", plan.lds_search,
                    plan.lds_merge);

    const size_t S = (size_t)n_inst * L;
    std::vector<long long> joff(n_inst);
    long long jtot = 0;
    for (int b = 0; b < n_inst; ++b) {
        joff[b] = jtot;
        jtot += (long long)N[b] * N[b];
    }
    BruteBufs buf;   // freed on every exit path
    int *dN = nullptr, *dborn = nullptr, *dexp = nullptr;
    long long* djoff = nullptr;
    double *dJ = nullptr, *dh = nullptr, *dE = nullptr, *dmE = nullptr;
    uint64_t *dx0 = nullptr, *dpsi = nullptr, *dmpsi = nullptr;
    uint8_t* dused = nullptr;
    if ((rc = buf.get(&dN, n_inst)) || (rc = buf.get(&djoff, n_inst)) || (rc = buf.get(&dJ, (size_t)jtot)) ||
        (rc = buf.get(&dh, (size_t)n_inst * 64)) || (rc = buf.get(&dx0, S)) || (rc = buf.get(&dpsi, S * K1)) ||
        (rc = buf.get(&dE, S * K1)) || (rc = buf.get(&dused, S * K1)) || (rc = buf.get(&dborn, S * K1)) ||
        (rc = buf.get(&dexp, S)) || (rc = buf.get(&dmpsi, (size_t)n_inst * K1)) || (rc = buf.get(&dmE, (size_t)n_inst * K1)))
        return rc;
    unsigned char* dws = nullptr;   // one region per search block (the merge blocks reuse the first ones)
    if (plan.ws_stride && (rc = buf.get(&dws, S * plan.ws_stride))) return rc;
    {
        std::vector<double> Jh((size_t)jtot), hh((size_t)n_inst * 64, 0.0);
        std::vector<uint64_t> xh(S);
        for (int b = 0; b < n_inst; ++b) {
            std::memcpy(Jh.data() + joff[b], J[b], sizeof(double) * N[b] * N[b]);
            std::memcpy(hh.data() + (size_t)b * 64, h[b], sizeof(double) * N[b]);
            for (int l = 0; l < L; ++l) xh[(size_t)b * L + l] = init_bits[b][l];
        }
        HIP_TRY(hipMemcpyAsync(dN, N, sizeof(int) * n_inst, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(djoff, joff.data(), sizeof(long long) * n_inst, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(dJ, Jh.data(), sizeof(double) * Jh.size(), hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(dh, hh.data(), sizeof(double) * hh.size(), hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(dx0, xh.data(), sizeof(uint64_t) * S, hipMemcpyHostToDevice, st));
        HIP_TRY(hipStreamSynchronize(st));
    }
    BestFirstArgs a{};
    a.L = L;
    a.K1 = K1;
    a.I = I;
    a.Cs = Cs;
    a.h1 = h1;
    a.N = dN;
    a.joff = djoff;
    a.J = dJ;
    a.h = dh;
    a.x0 = dx0;
    a.out_psi = dpsi;
    a.out_E = dE;
    a.out_used = dused;
    a.out_born = dborn;
    a.out_expanded = dexp;
    a.merged_psi = dmpsi;
    a.merged_E = dmE;
    a.lists_in_lds = plan.lists_in_lds;
    a.merge_in_lds = plan.merge_in_lds;
    a.ws = dws;
    a.ws_stride = plan.ws_stride;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (kernel_ms) {
        HIP_TRY(hipEventCreate(&e0));
        if (hipEventCreate(&e1) != hipSuccess) {
            (void)hipEventDestroy(e0);
            return fail(ISING_ERR_HIP, "hipEventCreate failed");
        }
        e = hipEventRecord(e0, st);
    }
    if (e == hipSuccess) e = launch_bestfirst(a, n_inst, plan, st);
    if (e == hipSuccess && kernel_ms) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess && kernel_ms) *kernel_ms = (float)elapsed_ms(e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) return fail(ISING_ERR_HIP, "best-first launch failed: %s", hipGetErrorString(e));
    // the real entries (E < +inf) in list order
    std::vector<uint64_t> mp((size_t)n_inst * K1);
    std::vector<double> mE((size_t)n_inst * K1);
    HIP_TRY(hipMemcpy(mp.data(), dmpsi, sizeof(uint64_t) * mp.size(), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(mE.data(), dmE, sizeof(double) * mE.size(), hipMemcpyDeviceToHost));
    for (int b = 0; b < n_inst; ++b) {
        int n = 0;
        for (int k = 0; k < K1; ++k) {
            const size_t q = (size_t)b * K1 + k;
            if (!(mE[q] < INFINITY)) break;
            merged_bits[(size_t)b * K1 + n] = mp[q];
            merged_E[(size_t)b * K1 + n] = mE[q];
            ++n;
        }
        merged_count[b] = n;
    }
    if (expanded) HIP_TRY(hipMemcpy(expanded, dexp, sizeof(int) * S, hipMemcpyDeviceToHost));
    if (search_bits || search_E || search_used || search_born || search_count) {
        if (!search_bits || !search_E || !search_count)
            return fail(ISING_ERR_INVALID_ARG, "search_bits, search_E and search_count go together");
        std::vector<uint64_t> sp(S * K1);
        std::vector<double> sE(S * K1);
        std::vector<uint8_t> su(S * K1);
        std::vector<int> sb(S * K1);
        HIP_TRY(hipMemcpy(sp.data(), dpsi, sizeof(uint64_t) * sp.size(), hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(sE.data(), dE, sizeof(double) * sE.size(), hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(su.data(), dused, su.size(), hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(sb.data(), dborn, sizeof(int) * sb.size(), hipMemcpyDeviceToHost));
        for (size_t q = 0; q < S; ++q) {
            int n = 0;
            for (int k = 0; k < K1; ++k) {
                const size_t o = q * K1 + k;
                if (!(sE[o] < INFINITY)) break;
                search_bits[q * K1 + n] = sp[o];
                search_E[q * K1 + n] = sE[o];
                if (search_used) search_used[q * K1 + n] = su[o];
                if (search_born) search_born[q * K1 + n] = sb[o];
                ++n;
            }
            search_count[q] = n;
        }
    }
    return ISING_OK;
}
