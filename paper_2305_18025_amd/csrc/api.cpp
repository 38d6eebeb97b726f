// Host side of the C ABI declared in include/pimdb.h: handle, argument
// validation, batch schedule, workspace accounting and kernel launches.
#include "../../include/pimdb.h"
#include "internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <vector>

using namespace pimdb;

namespace pimdb {
size_t exchange_smem_bytes(int threads);
}

struct pimdb_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    // batch definition
    int S = 0;
    std::vector<int64_t> N;
    std::vector<int32_t> P;
    std::vector<double> beta, m, omegaP;
    int64_t Nmax = 0;
    // derived tables (host copies and device copies)
    std::vector<SysDesc> desc;
    int64_t total_elems = 0;
    int64_t ws_doubles = 0; // after the header
    int64_t st_doubles = 0;
    SysDesc *d_desc = nullptr;
    Item *d_items = nullptr; // item lists back to back: [fb + sp | f + sp | b + sp | sp]
    int n_fb = 0, n_f = 0, n_b = 0, n_s = 0;
    EChunk *d_echunks = nullptr;
    int n_echunks = 0;
    // tables replaced after a call was captured into a graph: the graph
    // still reads them, so they are freed only by pimdb_destroy
    bool captured = false;
    std::vector<void *> retired;
    // optional HIP events around the two launches of an eager evaluation
    bool timing = false;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    bool ev_recorded = false;
    // settings
    double box = 0.0, trap_w = 0.0;
    int precision = PIMDB_FP64;
    int user_threads = 0, user_per = 0;
    int threads = 256, per_thread = 4;
    // split recursions: user setting (-1 automatic, 0 off, g >= 1 blocks per
    // helper) and what the current tables use
    int user_split = -1;
    int split_g = 0;       // 0: no system split
    int split_mode = 0;    // launch variant: 0 whole, 1 split, 2 split with a CU per workgroup
    int split_rows = 0;    // row waves per helper workgroup
    int helpers_total = 0; // helper workgroups of a forces launch
    int cus = 0;           // compute units of the device
    uint64_t wait_ticks = 200000000ull; // split waits give up after 2 s (100 MHz clock)
    // algorithm: the quadratic one, or the original cubic one (comparison
    // path) with its shift of the forward recurrence; the original one's
    // per-system workspace regions (offsets in doubles)
    int algorithm = PIMDB_ALG_FAST;
    int shift = PIMDB_SHIFT_MIN;
    std::vector<int64_t> orig_ws;
    int64_t orig_doubles = 0;
    // scaled pair interaction (g = 0: none): its work items, the first item
    // of each system, and the energy partials' offset in the workspace
    double pair_g = 0.0, pair_sigma = 1.0;
    PairItem *d_pitems = nullptr;
    int32_t *d_pbeg = nullptr;
    int n_pitems = 0, pair_iblock = 256;
    int64_t pair_off = 0;
    // workspace
    char *ws = nullptr;
    size_t ws_bytes = 0;
    // workspace whose header (status word) the last evaluation used: the
    // bound one, or the device's static scratch (pimdb_exchange_forces_static)
    char *status_ws = nullptr;
    std::string last_error;
};

// Scratch of pimdb_exchange_forces_static: a file-scope device array, one
// copy per device, held until the process ends.  Host code never passes
// `scratch` itself (in host code it names a host-side stand-in); it uses the
// device address that hipGetSymbolAddress returns for the current device,
// kept per device in g_scratch.
static __device__ __align__(256) unsigned char scratch[PIMDB_STATIC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch[MAX_DEVICES] = {};       // device address of `scratch` per device
hipError_t g_scratch_err[MAX_DEVICES] = {}; // why it could not be set up

// Once per device, with that device current: look up the device address of
// `scratch` and clear its status word (a kernel, then a wait: set-up only).
void scratch_setup(int dev) {
    if (dev < 0 || dev >= MAX_DEVICES) return;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch[dev] || g_scratch_err[dev] != hipSuccess) return;
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e == hipSuccess) e = launch_clear((int32_t *)p, PIMDB_STATIC_SCRATCH_BYTES / 4, nullptr);
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) {
        g_scratch_err[dev] = e;
        return;
    }
    g_scratch[dev] = p;
}

void *scratch_ptr(int dev) {
    if (dev < 0 || dev >= MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch[dev];
}

int fail(pimdb_t h, int code, const std::string &msg) {
    if (h) h->last_error = msg;
    return code;
}

int hip_fail(pimdb_t h, hipError_t e, const char *where) {
    return fail(h, PIMDB_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

struct DeviceGuard {
    int old = -1;
    bool ok = true;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&old) != hipSuccess) old = -1;
        if (old != dev) ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        int cur = -1;
        if (old >= 0 && hipGetDevice(&cur) == hipSuccess && cur != old) (void)hipSetDevice(old);
    }
};

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

bool pow2_threads(int t) { return t == 64 || t == 128 || t == 256 || t == 512 || t == 1024; }

int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// Automatic launch shape.  The recursion workgroups of the batch (two per
// system) should bring about 16 waves to every one of the 256 CUs: two
// particles per thread (more independent rows per lane) when that still
// reaches 4096 recursion waves, else the widest workgroup that holds the
// largest system with one particle per thread.  (Four rows per thread, in
// the 512-thread kernel with 3 waves per SIMD, measured slower than two at
// every batch size.)  Above 2048 particles only 512 threads x 8 rows fit
// the register budget.
void auto_tuning(int64_t Nmax, int S, int &threads, int &per) {
    if (Nmax > 2048) {
        threads = 512;
        per = 8;
        return;
    }
    auto width = [&](int p) {
        int64_t t = 64;
        while (t * p < Nmax) t *= 2;
        return t;
    };
    threads = (int)width(1);
    per = 1;
    if (threads > 1024) { // 1025..2048 particles
        threads = 1024;
        per = 2;
    }
    const int64_t t2 = width(2);
    if (2 * (int64_t)S * (t2 / 64) >= 4096) {
        threads = (int)t2;
        per = 2;
    }
}

// Split recursions (exchange.h): with lag L (2 when two workgroups share a
// CU, 3 when each has its own), a system of nblk = ceil(N / 64) > L blocks
// gets nhelp = ceil((nblk - L) / g) helper workgroups per direction, each
// owning at most g of the blocks L .. nblk-1 (forward; backward mirrored)
// on its row waves (rows per thread <= 2).  Systems of at most L blocks
// stay whole.  The launch must fit the workgroups the device holds at once,
// since the chain and helpers of a system wait on each other.
constexpr int SPLIT_T = 512;
// A helper's row waves: one per SIMD when every workgroup has a CU of its
// own (launch mode 2), all but the fetch wave when two share a CU (mode 1).
int split_rows(int mode) { return mode == 2 ? 4 : SPLIT_T / 64 - 1; }
// Threads of a split launch's workgroups: 1024 when each has a CU of its own
// (a chain's phase A on 16 waves), else 512 (two per CU).
int split_threads(int mode) { return mode == 2 ? 2 * SPLIT_T : SPLIT_T; }
// Blocks between a published block and the one a helper delivers from it:
// 3 when each workgroup has a CU (the chain forms the terms of the two
// blocks before its current one while the steps run), else 2.
int split_lag(int mode) { return mode == 2 ? 3 : 2; }

struct SplitPlan {
    int per = 1;
    int helpers = 0; // per forces launch (both directions)
    int recursion_wgs = 0;
    int mode = 1;    // 2: one workgroup per CU (the plan fits), 1: two per CU
    int rows = 7;    // a helper's row waves
    int threads = 512;
    std::vector<int> nhelp;
};

int helpers_for(int64_t N, int g, int rows, int lag) {
    const int nblk = (int)((N + 63) / 64);
    if (nblk <= lag || g < 1) return 0;
    int nh = (nblk - lag + g - 1) / g;
    const int most = 2 * rows; // blocks a helper can hold with two rows per thread
    nh = std::max(nh, (nblk - lag + most - 1) / most);
    return std::min(nh, nblk - lag);
}

// The plan for g blocks per helper: a CU of its own for every chain and
// helper when they all fit so (no SIMD shared with another workgroup, four
// row waves per helper), else two per CU (seven row waves).
bool plan_split(pimdb_t h, int g, SplitPlan &p) {
    const int S = h->S;
    const bool box = h->box > 0 || h->precision == PIMDB_FP64_DIRECT, mixed = h->precision == PIMDB_MIXED;
    for (int mode : {2, 1}) {
        const int rows = split_rows(mode), lag = split_lag(mode);
        p.nhelp.assign(S, 0);
        p.per = 1;
        p.helpers = 0;
        p.recursion_wgs = 0;
        for (int s = 0; s < S; ++s) {
            const int nblk = (int)((h->N[s] + 63) / 64);
            const int nh = helpers_for(h->N[s], g, rows, lag);
            p.nhelp[s] = nh;
            if (nh > 0) {
                const int own = (nblk - lag + nh - 1) / nh;
                p.per = std::max(p.per, (own + rows - 1) / rows);
            } else {
                p.per = std::max(p.per, (int)((h->N[s] + split_threads(mode) - 1) / split_threads(mode)));
            }
            p.helpers += 2 * nh;
            p.recursion_wgs += 2 + 2 * nh;
        }
        if (p.per > 2 || p.helpers == 0) continue;
        const int occ = exchange_occupancy(box, mixed, split_threads(mode), p.per, mode);
        if (occ > 0 && (int64_t)p.recursion_wgs <= (int64_t)occ * h->cus) {
            p.mode = mode;
            p.rows = rows;
            p.threads = split_threads(mode);
            return true;
        }
    }
    return false;
}

int auto_split(pimdb_t h, SplitPlan &p) {
    if (2 * (int64_t)h->S * 2 > h->cus) return 0;
    for (int g : {4, 7, 14, 28, 56}) {
        if (plan_split(h, g, p)) return g;
    }
    return 0;
}

// Release the current tables: freed at once, or kept until pimdb_destroy
// if a graph may hold them.
void free_tables(pimdb_t h, bool all = false) {
    for (void *p : {(void *)h->d_desc, (void *)h->d_items, (void *)h->d_echunks, (void *)h->d_pitems,
                    (void *)h->d_pbeg}) {
        if (!p) continue;
        if (h->captured && !all)
            h->retired.push_back(p);
        else
            (void)hipFree(p);
    }
    if (all) {
        for (void *p : h->retired) (void)hipFree(p);
        h->retired.clear();
    }
    h->d_desc = nullptr;
    h->d_items = nullptr;
    h->d_echunks = nullptr;
    h->d_pitems = nullptr;
    h->d_pbeg = nullptr;
    h->n_fb = h->n_f = h->n_b = h->n_s = h->n_echunks = h->n_pitems = 0;
}

// Build descriptors, the launch schedule (largest systems first) and the MD
// element chunks for the current batch and launch shape; upload them.
int build_tables(pimdb_t h) {
    // the workspace layout (per-system regions) depends on the
    // batch and the launch shape: the caller binds a workspace again
    h->ws = nullptr;
    h->ws_bytes = 0;
    h->status_ws = nullptr;
    DeviceGuard g(h->device);
    if (!g.ok) return fail(h, PIMDB_EDEVICE, "cannot select device");
    if (!h->cus) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess || n <= 0)
            return fail(h, PIMDB_EDEVICE, "cannot query the compute-unit count");
        h->cus = n;
    }
    // split recursions: the user's blocks per helper, or the automatic choice
    // (never with an explicit launch shape that is not the split one)
    SplitPlan plan;
    h->split_g = 0;
    if (h->user_split > 0) {
        if (!plan_split(h, h->user_split, plan))
            return fail(h, PIMDB_EINVAL, "this split does not fit the device (too many workgroups)");
        h->split_g = h->user_split;
    } else if (h->user_split < 0 && !h->user_threads) {
        h->split_g = auto_split(h, plan);
    }
    h->split_mode = h->split_g > 0 ? plan.mode : 0;
    h->split_rows = h->split_g > 0 ? plan.rows : 0;
    if (h->split_g > 0) {
        h->threads = plan.threads;
        h->per_thread = plan.per;
    } else if (h->user_threads) {
        h->threads = h->user_threads;
        h->per_thread = h->user_per;
    } else {
        auto_tuning(h->Nmax, h->S, h->threads, h->per_thread);
    }
    h->helpers_total = h->split_g > 0 ? plan.helpers : 0;
    const int T = h->threads;
    const int S = h->S;
    h->desc.assign(S, SysDesc{});
    int64_t off = 0, ws = 0, st = 0;
    for (int s = 0; s < S; ++s) {
        SysDesc &d = h->desc[s];
        d.off = off;
        d.ws = ws;
        d.st = st;
        d.N = (int32_t)h->N[s];
        d.P = h->P[s];
        d.nchunk = (int32_t)((h->N[s] + T - 1) / T);
        d.nhelp = h->split_g > 0 ? plan.nhelp[s] : 0;
        d.beta = h->beta[s];
        d.m = h->m[s];
        d.omegaP = h->omegaP[s];
        d.k = 0.5 * d.m * d.omegaP * d.omegaP;
        d.mw2 = d.m * d.omegaP * d.omegaP;
        d.kappa = -d.beta * d.k * 1.4426950408889634; // log2(e)
        off += (int64_t)3 * d.P * d.N;
        ws += round_up(WsLayout::total(d.N, d.nchunk), 32);
        st += round_up(StLayout::total(d.N), 32);
        d.xs = -1;
        if (d.nhelp > 0) {
            d.xs = ws;
            ws += round_up(XsLayout::total((d.N + 63) / 64), 32);
        }
    }
    h->total_elems = off;
    h->ws_doubles = ws;
    h->st_doubles = st;
    // the original algorithm's regions (only when it is selected: O(P N^2)
    // doubles per system); the two layouts share the workspace, which is
    // sized for the larger
    h->orig_ws.assign(S, 0);
    h->orig_doubles = 0;
    if (h->algorithm == PIMDB_ALG_ORIGINAL) {
        int64_t o = 0;
        for (int s = 0; s < S; ++s) {
            h->orig_ws[s] = o;
            o += round_up(OrigLayout::total(h->N[s], h->P[s]), 32);
        }
        h->orig_doubles = o;
    }
    // pair interaction items: every slice of every system in particle blocks
    // of the widest size that still gives 2048 workgroups (or 64)
    std::vector<PairItem> pit;
    std::vector<int32_t> pbeg;
    if (h->pair_g != 0.0) {
        int ib = 256;
        for (; ib > 64; ib /= 2) {
            int64_t n = 0;
            for (int s = 0; s < S; ++s) n += (int64_t)h->P[s] * ((h->N[s] + ib - 1) / ib);
            if (n >= 2048) break;
        }
        h->pair_iblock = ib;
        for (int s = 0; s < S; ++s) {
            pbeg.push_back((int32_t)pit.size());
            for (int j = 0; j < h->P[s]; ++j)
                for (int64_t i0 = 0; i0 < h->N[s]; i0 += ib) pit.push_back(PairItem{s, j, (int32_t)i0, 0});
        }
        pbeg.push_back((int32_t)pit.size());
    }

    // schedule: recursion items by decreasing N (forward and backward of a
    // system adjacent), then the spring items.
    std::vector<int> order(S);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return h->N[a] > h->N[b]; });
    // (split systems: both chains, then their helpers)
    std::vector<Item> fb, f, b, sp;
    for (int s : order) {
        fb.push_back(Item{s, ROLE_FORWARD, 0, 0});
        fb.push_back(Item{s, ROLE_BACKWARD, 0, 0});
        f.push_back(Item{s, ROLE_FORWARD, 0, 0});
        b.push_back(Item{s, ROLE_BACKWARD, 0, 0});
        for (int x = 0; x < h->desc[s].nhelp; ++x) {
            fb.push_back(Item{s, ROLE_FHELP, x, 0});
            fb.push_back(Item{s, ROLE_BHELP, x, 0});
            f.push_back(Item{s, ROLE_FHELP, x, 0});
            b.push_back(Item{s, ROLE_BHELP, x, 0});
        }
    }
    for (int s : order)
        for (int c = 0; c < h->desc[s].nchunk; ++c) sp.push_back(Item{s, ROLE_SPRINGS, c, 0});
    std::vector<Item> all;
    all.insert(all.end(), fb.begin(), fb.end());
    all.insert(all.end(), sp.begin(), sp.end());
    all.insert(all.end(), f.begin(), f.end());
    all.insert(all.end(), sp.begin(), sp.end());
    all.insert(all.end(), b.begin(), b.end());
    all.insert(all.end(), sp.begin(), sp.end());
    all.insert(all.end(), sp.begin(), sp.end());

    // MD update chunks: 8192 elements (32 per thread of a 256-thread
    // workgroup), so a batch of a few million elements still spreads over
    // several workgroups per CU (65536-element chunks left two thirds of the
    // CUs idle on the 64-system batch)
    std::vector<EChunk> ec;
    const int64_t CE = 1 << 13;
    for (int s = 0; s < S; ++s) {
        const int64_t b0 = h->desc[s].off, e0 = b0 + (int64_t)3 * h->desc[s].P * h->desc[s].N;
        for (int64_t x = b0; x < e0; x += CE) ec.push_back(EChunk{s, 0, x, std::min(e0, x + CE)});
    }

    free_tables(h);
    h->n_fb = (int)(fb.size() + sp.size());
    h->n_f = (int)(f.size() + sp.size());
    h->n_b = (int)(b.size() + sp.size());
    h->n_s = (int)sp.size();
    h->n_echunks = (int)ec.size();
    h->n_pitems = (int)pit.size();
    h->pair_off = std::max(h->ws_doubles, h->orig_doubles);
    hipError_t e;
    if ((e = hipMalloc(&h->d_desc, sizeof(SysDesc) * S)) != hipSuccess) return hip_fail(h, e, "hipMalloc");
    if ((e = hipMalloc(&h->d_items, sizeof(Item) * all.size())) != hipSuccess) return hip_fail(h, e, "hipMalloc");
    if ((e = hipMalloc(&h->d_echunks, sizeof(EChunk) * ec.size())) != hipSuccess) return hip_fail(h, e, "hipMalloc");
    if ((e = hipMemcpy(h->d_desc, h->desc.data(), sizeof(SysDesc) * S, hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(h, e, "hipMemcpy");
    if ((e = hipMemcpy(h->d_items, all.data(), sizeof(Item) * all.size(), hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(h, e, "hipMemcpy");
    if ((e = hipMemcpy(h->d_echunks, ec.data(), sizeof(EChunk) * ec.size(), hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(h, e, "hipMemcpy");
    if (!pit.empty()) {
        if ((e = hipMalloc(&h->d_pitems, sizeof(PairItem) * pit.size())) != hipSuccess) return hip_fail(h, e, "hipMalloc");
        if ((e = hipMalloc(&h->d_pbeg, sizeof(int32_t) * pbeg.size())) != hipSuccess) return hip_fail(h, e, "hipMalloc");
        if ((e = hipMemcpy(h->d_pitems, pit.data(), sizeof(PairItem) * pit.size(), hipMemcpyHostToDevice)) != hipSuccess)
            return hip_fail(h, e, "hipMemcpy");
        if ((e = hipMemcpy(h->d_pbeg, pbeg.data(), sizeof(int32_t) * pbeg.size(), hipMemcpyHostToDevice)) != hipSuccess)
            return hip_fail(h, e, "hipMemcpy");
    }
    return PIMDB_OK;
}

size_t ws_bytes_needed(pimdb_t h) {
    return (size_t)(WS_HEADER_BYTES + (std::max(h->ws_doubles, h->orig_doubles) + h->n_pitems) * 8);
}

int check_ready(pimdb_t h) {
    if (!h) return PIMDB_EINVAL;
    if (h->S <= 0) return fail(h, PIMDB_ENOSYS, "no system set");
    if (!h->ws || h->ws_bytes < ws_bytes_needed(h))
        return fail(h, PIMDB_EWORKSPACE, "workspace not bound or too small");
    return PIMDB_OK;
}

LaunchArgs base_args(pimdb_t h, char *ws) {
    LaunchArgs a{};
    a.sys = h->d_desc;
    a.flags = (int32_t *)ws;
    a.ws = (double *)(ws + WS_HEADER_BYTES);
    a.box = h->box;
    a.inv_box = h->box > 0 ? 1.0 / h->box : 0.0;
    a.trap_w2 = h->trap_w * h->trap_w;
    a.mixed = h->precision == PIMDB_MIXED;
    a.direct = h->precision == PIMDB_FP64_DIRECT;
    a.wait_ticks = h->wait_ticks;
    a.help_rows = h->split_rows;
    return a;
}

// Item list ranges inside d_items (see build_tables).
const Item *items_fb(pimdb_t h) { return h->d_items; }
const Item *items_f(pimdb_t h) { return h->d_items + h->n_fb; }
const Item *items_b(pimdb_t h) { return h->d_items + h->n_fb + h->n_f; }
const Item *items_s(pimdb_t h) { return h->d_items + h->n_fb + h->n_f + h->n_b; }

// The pair interaction on top of what an evaluation wrote (accumulate = 1),
// or alone; sign -1 with gscale: the adjoint's gradient.
hipError_t run_pair(pimdb_t h, char *ws, const double *pos, double *out, double *energy, const int64_t *offs,
                    const double *gscale, int sign, int accumulate) {
    if (h->pair_g == 0.0 || h->n_pitems == 0 || (!out && !energy)) return hipSuccess;
    PairArgs p{};
    p.sys = h->d_desc;
    p.items = h->d_pitems;
    p.beg = h->d_pbeg;
    p.offs = offs;
    p.pos = pos;
    p.out = out;
    p.energy = energy;
    p.epart = (double *)(ws + WS_HEADER_BYTES) + h->pair_off;
    p.gscale = gscale;
    p.flags = (int32_t *)ws;
    p.box = h->box;
    p.inv_box = h->box > 0 ? 1.0 / h->box : 0.0;
    p.c2 = -1.4426950408889634 / (2.0 * h->pair_sigma * h->pair_sigma);
    p.g = h->pair_g;
    p.inv_s2 = 1.0 / (h->pair_sigma * h->pair_sigma);
    p.sign = sign;
    p.accumulate = accumulate;
    p.iblock = h->pair_iblock;
    return launch_pair(p, h->n_pitems, h->S, h->stream);
}

int run(pimdb_t h, LaunchArgs &a, const Item *items, int n) {
    DeviceGuard g(h->device);
    if (!g.ok) return fail(h, PIMDB_EDEVICE, "cannot select device");
    h->status_ws = (char *)a.flags;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(h->stream, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) h->captured = true;
    const bool tm = h->timing && cs == hipStreamCaptureStatusNone;
    a.items = items;
    hipError_t e;
    if (tm && (e = hipEventRecord(h->ev[0], h->stream)) != hipSuccess) return hip_fail(h, e, "event");
    e = launch_exchange(a, n, h->threads, h->per_thread, h->split_mode, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "exchange launch");
    if (tm && (e = hipEventRecord(h->ev[1], h->stream)) != hipSuccess) return hip_fail(h, e, "event");
    e = launch_finalize(a, h->S, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "finalize launch");
    {
        const bool adj = (a.mode & M_ADJOINT) != 0;
        double *po = (a.mode & M_FORCES) ? a.out : nullptr;
        double *pe = (a.mode & M_ENERGY) ? a.energy : nullptr;
        e = run_pair(h, (char *)a.flags, a.pos, po, pe, a.offs, adj ? a.gscale : nullptr, adj ? -1 : 1, 1);
        if (e != hipSuccess) return hip_fail(h, e, "pair launch");
    }
    if (tm && (e = hipEventRecord(h->ev[2], h->stream)) != hipSuccess) return hip_fail(h, e, "event");
    h->ev_recorded = tm;
    return PIMDB_OK;
}

// The original algorithm, system after system (forces null: energy only).
int run_original(pimdb_t h, const double *pos, double *forces, double *energy) {
    DeviceGuard g(h->device);
    if (!g.ok) return fail(h, PIMDB_EDEVICE, "cannot select device");
    h->status_ws = h->ws;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(h->stream, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) h->captured = true;
    const bool tm = h->timing && cs == hipStreamCaptureStatusNone;
    hipError_t e;
    if (tm && (e = hipEventRecord(h->ev[0], h->stream)) != hipSuccess) return hip_fail(h, e, "event");
    for (int s = 0; s < h->S; ++s) {
        const SysDesc &d = h->desc[s];
        OrigArgs a{};
        a.pos = pos + d.off;
        a.out = forces ? forces + d.off : nullptr;
        a.energy = energy ? energy + s : nullptr;
        a.ws = (double *)(h->ws + WS_HEADER_BYTES) + h->orig_ws[s];
        a.flags = (int32_t *)h->ws;
        a.N = d.N;
        a.P = d.P;
        a.beta = d.beta;
        a.k = d.k;
        a.mw2 = d.mw2;
        a.box = h->box;
        a.inv_box = h->box > 0 ? 1.0 / h->box : 0.0;
        a.trapc = d.m * h->trap_w * h->trap_w / (double)d.P;
        a.two_term = h->shift == PIMDB_SHIFT_TWO_TERM;
        if ((e = launch_original(a, h->stream)) != hipSuccess) return hip_fail(h, e, "original algorithm launch");
    }
    if ((e = run_pair(h, h->ws, pos, forces, energy, nullptr, nullptr, 1, 1)) != hipSuccess)
        return hip_fail(h, e, "pair launch");
    if (tm) {
        if ((e = hipEventRecord(h->ev[1], h->stream)) != hipSuccess) return hip_fail(h, e, "event");
        if ((e = hipEventRecord(h->ev[2], h->stream)) != hipSuccess) return hip_fail(h, e, "event");
    }
    h->ev_recorded = tm;
    return PIMDB_OK;
}

int fast_only(pimdb_t h) {
    return h->algorithm == PIMDB_ALG_FAST ? PIMDB_OK
                                          : fail(h, PIMDB_EINVAL, "not available with the original algorithm");
}

int set_batch_impl(pimdb_t h, int32_t S, const int64_t *N, const int32_t *P, const double *beta,
                   const double *m, const double *omega_P) {
    if (!h) return PIMDB_EINVAL;
    if (S < 1 || !N || !P || !beta || !m || !omega_P) return fail(h, PIMDB_EINVAL, "bad batch arguments");
    if (S > PIMDB_MAX_BATCH) return fail(h, PIMDB_ERANGE, "batch too large");
    int64_t nmax = 0;
    for (int s = 0; s < S; ++s) {
        if (N[s] < 1) return fail(h, PIMDB_EINVAL, "N < 1");
        if (P[s] < 2) return fail(h, PIMDB_EINVAL, "P < 2");
        if (!finite_pos(beta[s]) || !finite_pos(m[s]) || !finite_pos(omega_P[s]))
            return fail(h, PIMDB_EINVAL, "beta, m and omega_P must be finite and positive");
        if (N[s] > PIMDB_MAX_N) return fail(h, PIMDB_ERANGE, "N above PIMDB_MAX_N");
        nmax = std::max<int64_t>(nmax, N[s]);
    }
    if (h->user_threads && (int64_t)h->user_threads * h->user_per < nmax)
        return fail(h, PIMDB_EINVAL, "tuning override too small for this batch");
    h->S = S;
    h->N.assign(N, N + S);
    h->P.assign(P, P + S);
    h->beta.assign(beta, beta + S);
    h->m.assign(m, m + S);
    h->omegaP.assign(omega_P, omega_P + S);
    h->Nmax = nmax;
    const int rc = build_tables(h);
    if (rc != PIMDB_OK) h->S = 0;
    return rc;
}

} // namespace

extern "C" {

int pimdb_create(pimdb_t *out, int device, void *stream) {
    if (!out) return PIMDB_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return PIMDB_EDEVICE;
    if (device < 0 || device >= count) return PIMDB_EINVAL;
    pimdb_t h = new (std::nothrow) pimdb_ctx();
    if (!h) return PIMDB_EDEVICE;
    h->device = device;
    h->stream = (hipStream_t)stream;
    // the split recursions' wait limit in microseconds (tests of the timeout
    // path shorten it so that waits give up at once)
    if (const char *w = std::getenv("PIMDB_SPLIT_WAIT_US")) {
        const long long us = std::atoll(w);
        if (us >= 0) h->wait_ticks = (uint64_t)us * 100;
    }
    {
        DeviceGuard g(device);
        if (!g.ok) {
            delete h;
            return PIMDB_EDEVICE;
        }
        scratch_setup(device);
    }
    *out = h;
    return PIMDB_OK;
}

int pimdb_destroy(pimdb_t h) {
    if (!h) return PIMDB_OK;
    {
        DeviceGuard g(h->device);
        (void)hipStreamSynchronize(h->stream);
        free_tables(h, true);
        for (hipEvent_t &e : h->ev)
            if (e) (void)hipEventDestroy(e);
    }
    delete h;
    return PIMDB_OK;
}

int pimdb_set_stream(pimdb_t h, void *stream) {
    if (!h) return PIMDB_EINVAL;
    h->stream = (hipStream_t)stream;
    return PIMDB_OK;
}

int pimdb_set_system(pimdb_t h, int64_t N, int32_t P, double beta, double m, double omega_P) {
    return set_batch_impl(h, 1, &N, &P, &beta, &m, &omega_P);
}

int pimdb_set_batch(pimdb_t h, int32_t S, const int64_t *N, const int32_t *P, const double *beta,
                    const double *m, const double *omega_P) {
    return set_batch_impl(h, S, N, P, beta, m, omega_P);
}

int pimdb_set_box(pimdb_t h, double L) {
    if (!h) return PIMDB_EINVAL;
    if (!std::isfinite(L) || L < 0) return fail(h, PIMDB_EINVAL, "box side must be finite and >= 0");
    h->box = L;
    return PIMDB_OK;
}

int pimdb_set_trap(pimdb_t h, double w) {
    if (!h) return PIMDB_EINVAL;
    if (!std::isfinite(w) || w < 0) return fail(h, PIMDB_EINVAL, "trap frequency must be finite and >= 0");
    h->trap_w = w;
    return PIMDB_OK;
}

int pimdb_set_precision(pimdb_t h, int mode) {
    if (!h) return PIMDB_EINVAL;
    if (mode != PIMDB_FP64 && mode != PIMDB_MIXED && mode != PIMDB_FP64_DIRECT)
        return fail(h, PIMDB_EINVAL, "unknown precision mode");
    h->precision = mode;
    return PIMDB_OK;
}

int pimdb_set_algorithm(pimdb_t h, int algorithm, int shift) {
    if (!h) return PIMDB_EINVAL;
    if (algorithm != PIMDB_ALG_FAST && algorithm != PIMDB_ALG_ORIGINAL)
        return fail(h, PIMDB_EINVAL, "unknown algorithm");
    if (shift != PIMDB_SHIFT_MIN && shift != PIMDB_SHIFT_TWO_TERM) return fail(h, PIMDB_EINVAL, "unknown shift");
    if (algorithm == PIMDB_ALG_FAST && shift != PIMDB_SHIFT_MIN)
        return fail(h, PIMDB_EINVAL, "the quadratic algorithm takes no shift (its sums carry their own exponents)");
    h->algorithm = algorithm;
    h->shift = shift;
    if (h->S > 0) return build_tables(h);
    return PIMDB_OK;
}

int pimdb_set_pair_gaussian(pimdb_t h, double g, double sigma) {
    if (!h) return PIMDB_EINVAL;
    if (!std::isfinite(g)) return fail(h, PIMDB_EINVAL, "pair strength must be finite");
    if (g != 0.0 && !finite_pos(sigma)) return fail(h, PIMDB_EINVAL, "pair width must be finite and positive");
    h->pair_g = g;
    h->pair_sigma = g != 0.0 ? sigma : 1.0;
    if (h->S > 0) return build_tables(h);
    return PIMDB_OK;
}

int pimdb_pair_forces(pimdb_t h, const double *pos, double *forces, double *energy) {
    int rc = check_ready(h);
    if (rc) return rc;
    if (!pos || (!forces && !energy)) return fail(h, PIMDB_EINVAL, "null pointer");
    if (pos == forces) return fail(h, PIMDB_EINVAL, "positions and forces alias");
    if (h->pair_g == 0.0) return fail(h, PIMDB_EINVAL, "no pair interaction set");
    DeviceGuard g(h->device);
    if (!g.ok) return fail(h, PIMDB_EDEVICE, "cannot select device");
    h->status_ws = h->ws;
    const hipError_t e = run_pair(h, h->ws, pos, forces, energy, nullptr, nullptr, 1, 0);
    if (e != hipSuccess) return hip_fail(h, e, "pair launch");
    return PIMDB_OK;
}

int pimdb_get_algorithm(pimdb_t h, int *algorithm, int *shift) {
    if (!h || !algorithm || !shift) return PIMDB_EINVAL;
    *algorithm = h->algorithm;
    *shift = h->shift;
    return PIMDB_OK;
}

int pimdb_set_tuning(pimdb_t h, int threads, int per_thread) {
    if (!h) return PIMDB_EINVAL;
    if (threads == 0 && per_thread == 0) {
        h->user_threads = h->user_per = 0;
    } else {
        if (!pow2_threads(threads)) return fail(h, PIMDB_EINVAL, "threads must be 64, 128, 256, 512 or 1024");
        if (per_thread != 1 && per_thread != 2 && per_thread != 4 && per_thread != 8)
            return fail(h, PIMDB_EINVAL, "per_thread must be 1, 2, 4 or 8");
        if (per_thread >= 4 && threads > 512) return fail(h, PIMDB_EINVAL, "per_thread 4 and 8 need threads <= 512");
        if (h->S > 0 && (int64_t)threads * per_thread < h->Nmax)
            return fail(h, PIMDB_EINVAL, "threads * per_thread below the largest N");
        h->user_threads = threads;
        h->user_per = per_thread;
    }
    if (h->S > 0) return build_tables(h);
    return PIMDB_OK;
}

int pimdb_set_timing(pimdb_t h, int enable) {
    if (!h) return PIMDB_EINVAL;
    DeviceGuard g(h->device);
    if (!g.ok) return fail(h, PIMDB_EDEVICE, "cannot select device");
    if (enable && !h->ev[0]) {
        for (hipEvent_t &e : h->ev) {
            const hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess) return hip_fail(h, r, "hipEventCreate");
        }
    }
    h->timing = enable != 0;
    h->ev_recorded = false;
    return PIMDB_OK;
}

int pimdb_last_timing(pimdb_t h, float *exchange_ms, float *finalize_ms) {
    if (!h || !exchange_ms || !finalize_ms) return PIMDB_EINVAL;
    if (!h->ev_recorded) return fail(h, PIMDB_ENOSYS, "no timed evaluation recorded");
    DeviceGuard g(h->device);
    hipError_t e;
    if ((e = hipEventSynchronize(h->ev[2])) != hipSuccess) return hip_fail(h, e, "event sync");
    if ((e = hipEventElapsedTime(exchange_ms, h->ev[0], h->ev[1])) != hipSuccess) return hip_fail(h, e, "event time");
    if ((e = hipEventElapsedTime(finalize_ms, h->ev[1], h->ev[2])) != hipSuccess) return hip_fail(h, e, "event time");
    return PIMDB_OK;
}

int pimdb_set_split(pimdb_t h, int blocks_per_helper) {
    if (!h) return PIMDB_EINVAL;
    if (blocks_per_helper < -1) return fail(h, PIMDB_EINVAL, "blocks per helper must be -1, 0 or positive");
    const int old = h->user_split;
    h->user_split = blocks_per_helper;
    if (h->S > 0) {
        const int rc = build_tables(h);
        if (rc != PIMDB_OK) {
            const std::string msg = h->last_error;
            h->user_split = old;
            (void)build_tables(h);
            h->last_error = msg;
            return rc;
        }
    }
    return PIMDB_OK;
}

int pimdb_get_split(pimdb_t h, int *blocks_per_helper, int *helpers, int *cu_per_workgroup) {
    if (!h || !blocks_per_helper || !helpers) return PIMDB_EINVAL;
    *blocks_per_helper = h->split_g;
    *helpers = h->helpers_total;
    if (cu_per_workgroup) *cu_per_workgroup = h->split_mode == 2 ? 1 : 0;
    return PIMDB_OK;
}

int pimdb_get_tuning(pimdb_t h, int *threads, int *per_thread) {
    if (!h || !threads || !per_thread) return PIMDB_EINVAL;
    *threads = h->threads;
    *per_thread = h->per_thread;
    return PIMDB_OK;
}

int64_t pimdb_system_offset(pimdb_t h, int32_t s) {
    if (!h || s < 0 || s >= h->S) return -1;
    return h->desc[s].off;
}

int64_t pimdb_total_elements(pimdb_t h) { return h ? h->total_elems : 0; }

size_t pimdb_workspace_bytes(pimdb_t h) {
    if (!h || h->S <= 0) return 0;
    return ws_bytes_needed(h);
}

size_t pimdb_state_bytes(pimdb_t h) {
    if (!h || h->S <= 0) return 0;
    return (size_t)h->st_doubles * 8;
}

int pimdb_bind_workspace(pimdb_t h, void *dev_ptr, size_t bytes) {
    if (!h) return PIMDB_EINVAL;
    if (!dev_ptr) return fail(h, PIMDB_EINVAL, "null workspace");
    if (((uintptr_t)dev_ptr) % 256) return fail(h, PIMDB_EINVAL, "workspace must be 256-byte aligned");
    if (h->S > 0 && bytes < ws_bytes_needed(h)) return fail(h, PIMDB_EWORKSPACE, "workspace too small");
    h->ws = (char *)dev_ptr;
    h->ws_bytes = bytes;
    h->status_ws = h->ws;
    DeviceGuard g(h->device);
    if (!g.ok) return fail(h, PIMDB_EDEVICE, "cannot select device");
    // the status word and the split recursions' flags start at zero
    const int64_t need = h->S > 0 ? (int64_t)ws_bytes_needed(h) : WS_HEADER_BYTES;
    const int64_t nints = std::min<int64_t>(need, (int64_t)bytes) / 4;
    hipError_t e = launch_clear((int32_t *)dev_ptr, nints, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "clear workspace");
    return PIMDB_OK;
}

int pimdb_exchange_energy(pimdb_t h, const double *pos, double *energy) {
    int rc = check_ready(h);
    if (rc) return rc;
    if (!pos || !energy) return fail(h, PIMDB_EINVAL, "null pointer");
    if (h->algorithm == PIMDB_ALG_ORIGINAL) return run_original(h, pos, nullptr, energy);
    LaunchArgs a = base_args(h, h->ws);
    a.pos = pos;
    a.energy = energy;
    a.mode = M_FWD | M_ENERGY;
    return run(h, a, items_f(h), h->n_f);
}

int pimdb_exchange_forces(pimdb_t h, const double *pos, double *forces, double *energy) {
    int rc = check_ready(h);
    if (rc) return rc;
    if (!pos || !forces) return fail(h, PIMDB_EINVAL, "null pointer");
    if (pos == forces) return fail(h, PIMDB_EINVAL, "positions and forces alias");
    if (h->algorithm == PIMDB_ALG_ORIGINAL) return run_original(h, pos, forces, energy);
    LaunchArgs a = base_args(h, h->ws);
    a.pos = pos;
    a.out = forces;
    a.energy = energy;
    a.mode = M_FWD | M_BWD | M_WSUM | M_FORCES | (energy ? M_ENERGY : 0);
    return run(h, a, items_fb(h), h->n_fb);
}

int pimdb_exchange_forces_batched(pimdb_t h, const double *pos_packed, const int64_t *offsets_dev,
                                  double *forces_packed, double *energies) {
    int rc = check_ready(h);
    if (rc) return rc;
    if ((rc = fast_only(h))) return rc;
    if (!pos_packed || !offsets_dev || !forces_packed || !energies) return fail(h, PIMDB_EINVAL, "null pointer");
    if (pos_packed == forces_packed) return fail(h, PIMDB_EINVAL, "positions and forces alias");
    LaunchArgs a = base_args(h, h->ws);
    a.pos = pos_packed;
    a.out = forces_packed;
    a.energy = energies;
    a.offs = offsets_dev;
    a.mode = M_FWD | M_BWD | M_WSUM | M_FORCES | M_ENERGY;
    return run(h, a, items_fb(h), h->n_fb);
}

int pimdb_exchange_forces_static(pimdb_t h, const double *pos, double *forces, double *energy) {
    if (!h) return PIMDB_EINVAL;
    if (h->S <= 0) return fail(h, PIMDB_ENOSYS, "no system set");
    if (fast_only(h)) return PIMDB_EINVAL;
    if (!pos || !forces) return fail(h, PIMDB_EINVAL, "null pointer");
    if (pos == forces) return fail(h, PIMDB_EINVAL, "positions and forces alias");
    const size_t need = ws_bytes_needed(h);
    if (need > (size_t)PIMDB_STATIC_SCRATCH_BYTES)
        return fail(h, PIMDB_ERANGE, "batch needs " + std::to_string(need) +
                                         " bytes of scratch; the static scratch holds " +
                                         std::to_string((size_t)PIMDB_STATIC_SCRATCH_BYTES));
    char *ws = (char *)scratch_ptr(h->device);
    if (!ws) {
        const hipError_t e = (h->device >= 0 && h->device < MAX_DEVICES) ? g_scratch_err[h->device] : hipErrorInvalidDevice;
        return fail(h, PIMDB_EDEVICE, std::string("static scratch unavailable: ") + hipGetErrorString(e));
    }
    LaunchArgs a = base_args(h, ws);
    a.pos = pos;
    a.out = forces;
    a.energy = energy;
    a.mode = M_FWD | M_BWD | M_WSUM | M_FORCES | (energy ? M_ENERGY : 0);
    if (h->split_g > 0) { // the scratch holds the last call's contents, maybe of another layout
        DeviceGuard g(h->device);
        const hipError_t e = launch_clear_flags(a, h->S, h->stream);
        if (e != hipSuccess) return hip_fail(h, e, "clear flags");
    }
    return run(h, a, items_fb(h), h->n_fb);
}

int pimdb_exchange_energy_save(pimdb_t h, const double *pos, double *energy, void *state) {
    int rc = check_ready(h);
    if (rc) return rc;
    if ((rc = fast_only(h))) return rc;
    if (!pos || !energy || !state) return fail(h, PIMDB_EINVAL, "null pointer");
    LaunchArgs a = base_args(h, h->ws);
    a.pos = pos;
    a.energy = energy;
    a.state = (double *)state;
    a.mode = M_FWD | M_WSUM | M_SAVE | M_ENERGY;
    return run(h, a, items_f(h), h->n_f);
}

int pimdb_exchange_adjoint(pimdb_t h, const double *pos, const void *state, const double *grad_energy,
                           double *grad_pos) {
    int rc = check_ready(h);
    if (rc) return rc;
    if ((rc = fast_only(h))) return rc;
    if (!pos || !state || !grad_energy || !grad_pos) return fail(h, PIMDB_EINVAL, "null pointer");
    if (pos == grad_pos) return fail(h, PIMDB_EINVAL, "positions and gradient alias");
    LaunchArgs a = base_args(h, h->ws);
    a.pos = pos;
    a.out = grad_pos;
    a.state = (double *)state;
    a.gscale = grad_energy;
    a.mode = M_BWD | M_FORCES | M_ADJOINT;
    return run(h, a, items_b(h), h->n_b);
}

int pimdb_md_step(pimdb_t h, double *pos, double *vel, double *forces, double *energy, double dt) {
    int rc = check_ready(h);
    if (rc) return rc;
    if (!pos || !vel || !forces) return fail(h, PIMDB_EINVAL, "null pointer");
    if (!std::isfinite(dt)) return fail(h, PIMDB_EINVAL, "dt must be finite");
    DeviceGuard g(h->device);
    if (!g.ok) return fail(h, PIMDB_EDEVICE, "cannot select device");
    hipError_t e = launch_md_update(h->d_desc, h->d_echunks, h->n_echunks, pos, vel, forces, dt, 1, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "md kick/drift");
    rc = pimdb_exchange_forces(h, pos, forces, energy);
    if (rc) return rc;
    e = launch_md_update(h->d_desc, h->d_echunks, h->n_echunks, pos, vel, forces, dt, 0, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "md kick");
    return PIMDB_OK;
}

int pimdb_distinguishable_forces(pimdb_t h, const double *pos, double *forces, double *energy) {
    int rc = check_ready(h);
    if (rc) return rc;
    if (!pos || !forces) return fail(h, PIMDB_EINVAL, "null pointer");
    if (pos == forces) return fail(h, PIMDB_EINVAL, "positions and forces alias");
    LaunchArgs a = base_args(h, h->ws);
    a.pos = pos;
    a.out = forces;
    a.energy = energy;
    a.mode = M_DIST | M_FORCES | (energy ? M_ENERGY : 0);
    return run(h, a, items_s(h), h->n_s);
}

int pimdb_debug_get(pimdb_t h, const double *pos, int32_t s, int what, double *dst) {
    int rc = check_ready(h);
    if (rc) return rc;
    if (!pos || !dst) return fail(h, PIMDB_EINVAL, "null pointer");
    if (s < 0 || s >= h->S) return fail(h, PIMDB_EINVAL, "system index out of range");
    if (what < PIMDB_DEBUG_PROBABILITIES || what > PIMDB_DEBUG_BACKWARD)
        return fail(h, PIMDB_EINVAL, "unknown debug export");
    // recursions of the whole batch without force output
    LaunchArgs a = base_args(h, h->ws);
    a.pos = pos;
    a.mode = M_FWD | M_BWD | M_WSUM;
    if ((rc = run(h, a, items_fb(h), h->n_fb))) return rc;
    DeviceGuard g(h->device);
    hipError_t e;
    if (what != PIMDB_DEBUG_PROBABILITIES) {
        if ((e = launch_debug_prefix(a, s, h->threads, h->stream)) != hipSuccess)
            return hip_fail(h, e, "debug prefix");
    }
    if ((e = launch_debug_table(a, s, (int)h->N[s], what, dst, h->stream)) != hipSuccess)
        return hip_fail(h, e, "debug table");
    if ((e = hipStreamSynchronize(h->stream)) != hipSuccess) return hip_fail(h, e, "synchronize");
    return PIMDB_OK;
}

int pimdb_endpoint_springs(pimdb_t h, const double *pos, int32_t s, int as_float, void *dst) {
    if (!h) return PIMDB_EINVAL;
    if (h->S <= 0) return fail(h, PIMDB_ENOSYS, "no system set");
    if (!pos || !dst) return fail(h, PIMDB_EINVAL, "null pointer");
    if (s < 0 || s >= h->S) return fail(h, PIMDB_EINVAL, "system index out of range");
    LaunchArgs a = base_args(h, h->ws);
    a.pos = pos;
    DeviceGuard g(h->device);
    hipError_t e = launch_endpoint_springs(a, s, (int)h->N[s], as_float ? 1 : 0, dst, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "endpoint springs");
    return PIMDB_OK;
}

int pimdb_status(pimdb_t h, int32_t *flags) {
    if (!h) return PIMDB_EINVAL;
    char *sw = h->status_ws ? h->status_ws : h->ws;
    if (!sw) return fail(h, PIMDB_EWORKSPACE, "workspace not bound");
    DeviceGuard g(h->device);
    hipError_t e;
    if ((e = hipStreamSynchronize(h->stream)) != hipSuccess) return hip_fail(h, e, "synchronize");
    int32_t v = 0;
    if ((e = hipMemcpy(&v, sw, sizeof(v), hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(h, e, "read status");
    if ((e = launch_clear((int32_t *)sw, 1, h->stream)) != hipSuccess) return hip_fail(h, e, "clear status");
    if ((e = hipStreamSynchronize(h->stream)) != hipSuccess) return hip_fail(h, e, "synchronize");
    if (flags) *flags = v;
    return v ? PIMDB_ENONFINITE : PIMDB_OK;
}

const char *pimdb_strerror(int code) {
    switch (code) {
    case PIMDB_OK: return "success";
    case PIMDB_EINVAL: return "invalid argument";
    case PIMDB_ENOSYS: return "no system set";
    case PIMDB_EWORKSPACE: return "workspace missing or too small";
    case PIMDB_EDEVICE: return "HIP device error";
    case PIMDB_ENONFINITE: return "non-finite input or result (device status set)";
    case PIMDB_ERANGE: return "size out of supported range";
    default: return "unknown error";
    }
}

const char *pimdb_last_error(pimdb_t h) { return h ? h->last_error.c_str() : ""; }

} // extern "C"
