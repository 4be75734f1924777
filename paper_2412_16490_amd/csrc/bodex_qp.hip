// bodex_qp.hip -- host side of the C ABI declared in include/bodex_qp.h.
//
// Responsibilities: argument validation (host-side, before any device work),
// the tile schedule (which grasps share a wavefront), library-owned device
// workspace within the handle's budget, kernel launches on the handle's
// stream, and hipGraph capture/replay of repeated launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/bodex_qp.h"
#include "bodex_kernels.h"
#include "bodex_launch.h"

using bodex::KArgs;

// Scratch of the allocation-free solve (bodex_qp_solve_static): the batch
// descriptor the kernels read (contact counts, wrench offsets, tile order,
// tile starts, queue counters).  One copy per GPU, held until the process
// ends.  In host code this name stands for no device address: the device
// address of each GPU's copy comes from hipGetSymbolAddress (static_scratch).
static __device__ __align__(256) int scratch[BODEX_STATIC_SCRATCH_INTS];

namespace {

thread_local std::string g_create_error;

struct GraphEntry {
    uint64_t key = 0;
    hipGraphExec_t exec = nullptr;
    int* d_desc = nullptr;
    size_t desc_ints = 0;
    int* d_queue = nullptr;
    uint64_t stamp = 0;
};

struct Schedule {
    std::vector<int> perm;
    std::vector<int> tile_start;
    int slots = 1;
    int n_tiles = 0;
};

}  // namespace

struct bodex_qp {
    bodex_qp_params prm;
    int device = 0;
    hipStream_t stream = nullptr;
    size_t budget = 0;
    int n_cu = 256;
    std::string err;

    // device descriptor buffer: counts | woff | perm | tile_start | queue(4)
    int* d_desc = nullptr;
    size_t d_desc_cap = 0;
    int* h_desc = nullptr;  // pinned staging
    size_t h_desc_cap = 0;
    hipEvent_t desc_ev = nullptr;
    bool desc_pending = false;
    // internal state when the caller passes none
    float* d_state = nullptr;
    size_t d_state_cap = 0;
    // descent workspace: contacts, their gradients, distances, loss weights
    float* d_hand = nullptr;
    size_t d_hand_cap = 0;
    // chunked polish: spill records (doubles, then ints) and the record of each QP
    void* d_spill = nullptr;
    size_t d_spill_cap = 0;
    // graphs
    std::vector<GraphEntry> graphs;
    uint64_t graph_clock = 0;
    // stats of the last call
    int last_launches = 0, last_replays = 0, last_tiles = 0;
    size_t owned_bytes = 0;
    // timing events: admm begin/end, finalize begin/end, backward begin/end
    hipEvent_t tev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    bool t_admm = false, t_fin = false, t_bwd = false;
};

namespace {

int fail(bodex_qp* h, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (h)
        h->err = buf;
    else
        g_create_error = buf;
    return code;
}

int hip_fail(bodex_qp* h, hipError_t e, const char* what) {
    return fail(h, BODEX_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(h, call)                                   \
    do {                                                   \
        hipError_t e_ = (call);                            \
        if (e_ != hipSuccess) return hip_fail((h), e_, #call); \
    } while (0)

bool aligned4(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 3u) == 0; }

// Device address of `scratch` on each GPU (taken once per device with that
// device current), and the pageable host buffer the descriptor is staged in.
constexpr int kStaticMaxDevices = 64;
std::mutex g_static_mu;
int* g_static_dev[kStaticMaxDevices] = {};
int g_static_host[BODEX_STATIC_SCRATCH_INTS];

// With h->device current: this device's address of `scratch`.
int static_scratch(bodex_qp* h, int device, int** out) {
    if (device < 0 || device >= kStaticMaxDevices)
        return fail(h, BODEX_EUNSUP, "device %d: the static scratch covers devices 0..%d", device,
                    kStaticMaxDevices - 1);
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (!g_static_dev[device]) {
        void* ptr = nullptr;
        HIP_TRY(h, hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(h, BODEX_EHIP, "hipGetSymbolAddress returned NULL for the static scratch");
        g_static_dev[device] = static_cast<int*>(ptr);
    }
    *out = g_static_dev[device];
    return 0;
}

// Contact counts the kernels are compiled for.  A batch with m_max contacts
// per grasp runs on the smallest compiled size >= m_max (array strides stay
// m_max; the extra contacts are inert padding).  The circular cone's polish
// factors a dense 3 m x 3 m matrix per lane and is compiled up to 5.
constexpr int kCompiledMM[] = {4, 5, 6, 7, 8};
constexpr int kConeMaxMM = 5;

int kernel_mm(int m_max) {
    for (int mm : kCompiledMM)
        if (mm >= m_max) return mm;
    return 0;
}

size_t admm_lds(int mm, int slots) {
    switch (mm) {
        case 4: return bodex::AdmmLds<4>::bytes(slots);
        case 5: return bodex::AdmmLds<5>::bytes(slots);
        case 6: return bodex::AdmmLds<6>::bytes(slots);
        case 7: return bodex::AdmmLds<7>::bytes(slots);
        case 8: return bodex::AdmmLds<8>::bytes(slots);
    }
    return 0;
}

size_t fin_lds(int mm, int slots, bool bwd) {
    switch (mm) {
        case 4: return bodex::FinLds<4>::bytes(slots, bwd);
        case 5: return bodex::FinLds<5>::bytes(slots, bwd);
        case 6: return bodex::FinLds<6>::bytes(slots, bwd);
        case 7: return bodex::FinLds<7>::bytes(slots, bwd);
        case 8: return bodex::FinLds<8>::bytes(slots, bwd);
    }
    return 0;
}

// Build the tile schedule.  Plain: grasps in index order, greedily packed.
// Batched: grasps sorted by (m, s) so that tiles are uniform in contact count
// and pack wrench counts tightly; tiles ordered by estimated cost (largest
// first) for the persistent work queue.
void build_schedule(const int* counts, const int* woff, int G, bool batched, Schedule& S) {
    S.perm.resize(G);
    std::iota(S.perm.begin(), S.perm.end(), 0);
    if (batched) {
        std::stable_sort(S.perm.begin(), S.perm.end(), [&](int a, int b) {
            if (counts[a] != counts[b]) return counts[a] > counts[b];
            return (woff[a + 1] - woff[a]) > (woff[b + 1] - woff[b]);
        });
    }
    S.tile_start.clear();
    S.tile_start.push_back(0);
    int cur_q = 0, cur_n = 0, slots = 1;
    int cur_m = -1;
    for (int i = 0; i < G; ++i) {
        const int g = S.perm[i];
        const int s = woff[g + 1] - woff[g];
        const bool split = cur_n > 0 && (cur_q + s > bodex::kWave || cur_n >= bodex::kMaxSlots ||
                                         (batched && counts[g] != cur_m));
        if (split) {
            S.tile_start.push_back(i);
            slots = std::max(slots, cur_n);
            cur_q = 0;
            cur_n = 0;
        }
        cur_q += s;
        cur_n += 1;
        cur_m = counts[g];
    }
    if (cur_n > 0) {
        S.tile_start.push_back(G);
        slots = std::max(slots, cur_n);
    }
    S.n_tiles = int(S.tile_start.size()) - 1;
    S.slots = slots;
    if (batched && S.n_tiles > 1) {
        // largest tiles first: cost ~ m^2 * (QPs in tile)
        std::vector<int> order(S.n_tiles);
        std::iota(order.begin(), order.end(), 0);
        std::vector<long> cost(S.n_tiles);
        for (int t = 0; t < S.n_tiles; ++t) {
            long c = 0;
            for (int i = S.tile_start[t]; i < S.tile_start[t + 1]; ++i) {
                const int g = S.perm[i];
                c += long(counts[g]) * counts[g] * (woff[g + 1] - woff[g]);
            }
            cost[t] = c;
        }
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
        std::vector<int> perm2;
        std::vector<int> ts2{0};
        perm2.reserve(G);
        for (int t : order) {
            for (int i = S.tile_start[t]; i < S.tile_start[t + 1]; ++i) perm2.push_back(S.perm[i]);
            ts2.push_back(int(perm2.size()));
        }
        S.perm.swap(perm2);
        S.tile_start.swap(ts2);
    }
}

uint64_t fnv1a(uint64_t h, const void* p, size_t n) {
    const unsigned char* b = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) {
        h ^= b[i];
        h *= 1099511628211ull;
    }
    return h;
}

void drop_graphs(bodex_qp* h) {
    for (auto& g : h->graphs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.d_desc) (void)hipFree(g.d_desc);
        h->owned_bytes -= g.desc_ints * sizeof(int);
    }
    h->graphs.clear();
}

int ensure_device(bodex_qp* h, void** ptr, size_t* cap, size_t need) {
    if (*cap >= need) return 0;
    // captured graphs hold the old pointers
    if (!h->graphs.empty()) {
        HIP_TRY(h, hipStreamSynchronize(h->stream));
        drop_graphs(h);
    }
    size_t extra = need - *cap;
    if (h->owned_bytes + extra > h->budget)
        return fail(h, BODEX_EBUDGET, "workspace of %zu bytes exceeds the budget of %zu bytes",
                    h->owned_bytes + extra, h->budget);
    if (*ptr) {
        HIP_TRY(h, hipStreamSynchronize(h->stream));
        HIP_TRY(h, hipFree(*ptr));
        h->owned_bytes -= *cap;
        *ptr = nullptr;
        *cap = 0;
    }
    HIP_TRY(h, hipMalloc(ptr, need));
    *cap = need;
    h->owned_bytes += need;
    return 0;
}

// The cached graph for `key`, or a new entry (descriptor buffer of n_ints
// allocated, exec still null: the caller captures it).  At most 8 graphs are
// kept; the least recently launched one makes room.
int graph_entry(bodex_qp* h, uint64_t key, size_t n_ints, GraphEntry** out) {
    for (auto& g : h->graphs)
        if (g.key == key && g.exec) {
            *out = &g;
            return 0;
        }
    // a failed capture may have left an entry without a graph
    for (size_t i = 0; i < h->graphs.size(); ++i)
        if (!h->graphs[i].exec) {
            if (h->graphs[i].d_desc) HIP_TRY(h, hipFree(h->graphs[i].d_desc));
            h->owned_bytes -= h->graphs[i].desc_ints * sizeof(int);
            h->graphs.erase(h->graphs.begin() + i);
            break;
        }
    if (h->graphs.size() >= 8) {
        auto oldest = std::min_element(h->graphs.begin(), h->graphs.end(),
                                       [](const GraphEntry& x, const GraphEntry& y) { return x.stamp < y.stamp; });
        HIP_TRY(h, hipStreamSynchronize(h->stream));
        if (oldest->exec) HIP_TRY(h, hipGraphExecDestroy(oldest->exec));
        if (oldest->d_desc) HIP_TRY(h, hipFree(oldest->d_desc));
        h->owned_bytes -= oldest->desc_ints * sizeof(int);
        h->graphs.erase(oldest);
    }
    GraphEntry e;
    e.key = key;
    e.desc_ints = n_ints;
    if (h->owned_bytes + n_ints * sizeof(int) > h->budget)
        return fail(h, BODEX_EBUDGET, "graph descriptors exceed the budget");
    HIP_TRY(h, hipMalloc(reinterpret_cast<void**>(&e.d_desc), n_ints * sizeof(int)));
    h->owned_bytes += n_ints * sizeof(int);
    h->graphs.push_back(e);
    *out = &h->graphs.back();
    return 0;
}

enum class Kind { Admm, Fin, Bwd };

constexpr int kDefaultAdmmWaves = 2;
// polish_chunk -1 (the default): the chunk by batch size.  Measured at 256
// to 8192 grasps x 16 wrenches (5 contacts): the contact-parallel polish
// alone (chunk 1) is 2.8x faster than the one-lane polish at 256 grasps,
// 1.9x at 1024 and 1.4x at 2048, where its latency wins; from 4096 grasps
// the one-lane pass is needed for throughput, and a budget of 16
// factorisations (with the wavefront hand-off and the contact-parallel
// kernel at two waves per SIMD) is the fastest measured at 4096, 8192 and
// 16,384 grasps and level with 20 at 32,768.
constexpr int kDefaultPolishChunk = -1;
int auto_polish_chunk(int n_qps) { return n_qps <= 40960 ? 1 : 16; }
// ADMM stopping rule with the polish on, per friction model (admm_tol 0).
// The pyramid's active-set polish costs the same from a rough point: 1e-1.
// The cone's barrier polish is faster from a closer one (headline batch:
// finalize 19.7 ms from 1e-2, 12.5 ms from 1e-4 or tighter); the few QPs
// that take hundreds of iterations to get there hold up their whole grasp,
// so the cone's ADMM also stops at 200 iterations (ADMM 0.8 ms instead of
// 1.9 ms at 500, finalize unchanged).
constexpr float kAdmmTolPyramid = 1e-1f, kAdmmTolCone = 1e-4f;
constexpr int kAdmmItersCone = 200;
// The pyramid's ADMM under that rule is only a warm start, checked first
// after 20 iterations rather than 10: the polish from the 20-iteration point
// is faster by more than the extra iterations cost (headline batch, ADMM +
// polish: 1.87-1.90 ms against 1.95-1.99 ms).
constexpr int kAdmmCheckPyramid = 20;

// The rules the parameters leave to the library: ADMM's stopping
// tolerance, iteration cap and check period (with the polish on and
// admm_tol 0, the friction model's rule), and the polish's factorisation
// budget for a batch of n_qps QPs.
struct Effective {
    float admm_tol;
    int max_iters, check_every, polish_chunk;
};
Effective effective(const bodex_qp_params& p, int n_qps) {
    const bool cone_model = p.friction_cone == BODEX_CONE_CIRCULAR;
    const bool polish = (p.flags & BODEX_F_POLISH) != 0;
    const bool model_rule = polish && !(p.admm_tol > 0.f);
    Effective e;
    // without the polish nothing lifts a QP past the ADMM tolerance
    e.admm_tol = !polish ? p.tol_rel : (p.admm_tol > 0.f ? p.admm_tol : (cone_model ? kAdmmTolCone : kAdmmTolPyramid));
    e.max_iters = (model_rule && cone_model) ? std::min(p.max_iters, kAdmmItersCone) : p.max_iters;
    e.check_every = (model_rule && !cone_model) ? std::max(p.check_every, kAdmmCheckPyramid) : p.check_every;
    const bool chunkable = polish && !cone_model && p.gamma == 0.f;
    e.polish_chunk = !chunkable ? 0 : (p.polish_chunk < 0 ? auto_polish_chunk(n_qps) : p.polish_chunk);
    return e;
}

hipError_t launch(Kind k, int mm, const KArgs& a, int grid, size_t lds, hipStream_t st, int occ = 0) {
    if (k == Kind::Admm) return bodex::launch_admm(mm, occ > 0 ? occ : kDefaultAdmmWaves, a, grid, lds, st);
    if (k == Kind::Fin)
        return a.cone ? bodex::launch_finalize_cone(mm, a, grid, lds, st) : bodex::launch_finalize(mm, a, grid, lds, st);
    return a.cone ? bodex::launch_backward_cone(mm, a, grid, lds, st) : bodex::launch_backward(mm, a, grid, lds, st);
}

// Chunked polish (the factorisation budget polish_chunk, -1: by batch
// size): the one-lane pass hands QPs that need more factorisations to the
// contact-parallel polish.  Sets up the record workspace (records for every
// QP of the batch, so none is ever finished in the first pass for want of
// room) in a; chunked is false where the chunked polish does not apply (no
// polish, the circular cone, gamma > 0, chunk 0: effective()).
int chunk_setup(bodex_qp* h, KArgs& a, int W, int mm, bool& chunked, int& grid_g) {
    const int chunk = effective(h->prm, W).polish_chunk;
    chunked = chunk > 0;
    grid_g = 0;
    if (!chunked) return 0;
    const size_t K = size_t(W);
    const size_t nd = size_t(3 * mm + 3) * K, ni = size_t(bodex::kSpInts) * K + size_t(W);
    const int rc = ensure_device(h, &h->d_spill, &h->d_spill_cap, nd * sizeof(double) + ni * sizeof(int));
    if (rc) return rc;
    a.spill.d = static_cast<double*>(h->d_spill);
    a.spill.i = reinterpret_cast<int*>(a.spill.d + nd);
    a.spill.K = int(K);
    a.spill_idx = a.spill.i + size_t(bodex::kSpInts) * K;
    a.polish_budget = chunk;
    const int gpw = bodex::kWave / bodex::gpolish_group(mm);
    grid_g = int((K + gpw - 1) / gpw);
    return 0;
}

// The finalize launches: one, or for the chunked polish the budgeted first
// pass, the contact-parallel polish of what it handed on and the outputs of
// those QPs (the record counter is the second word of the queue counters,
// which the step's reset clears).
int enqueue_finalize(bodex_qp* h, KArgs f, int mm, bool chunked, int* d_queue, int grid_f, int grid_g,
                     size_t lds_f) {
    f.queue = nullptr;
    if (chunked) {
        f.spill_count = d_queue + 1;
        f.fin_mode = 1;
        HIP_TRY(h, launch(Kind::Fin, mm, f, grid_f, lds_f, h->stream));
        HIP_TRY(h, bodex::launch_gpolish(mm, f, grid_g, h->stream));
        f.fin_mode = 2;
        HIP_TRY(h, launch(Kind::Fin, mm, f, grid_f, lds_f, h->stream));
    } else {
        HIP_TRY(h, launch(Kind::Fin, mm, f, grid_f, lds_f, h->stream));
    }
    return 0;
}

int validate_params(const bodex_qp_params* p, bodex_qp* h) {
    if (!p) return fail(h, BODEX_EINVAL, "params is NULL");
    if (p->m_max < 1 || p->m_max > BODEX_MAX_CONTACTS)
        return fail(h, BODEX_EINVAL, "m_max=%d outside [1, %d]", p->m_max, BODEX_MAX_CONTACTS);
    if (p->s_max < 1 || p->s_max > BODEX_MAX_WRENCHES)
        return fail(h, BODEX_EINVAL, "s_max=%d outside [1, %d]", p->s_max, BODEX_MAX_WRENCHES);
    if (!(p->force_max > 0.f) || !std::isfinite(p->force_max))
        return fail(h, BODEX_EINVAL, "force_max must be positive");
    if (!(p->gamma >= 0.f) || !std::isfinite(p->gamma)) return fail(h, BODEX_EINVAL, "gamma must be >= 0");
    if (!(p->beta >= 0.f) || !std::isfinite(p->beta)) return fail(h, BODEX_EINVAL, "beta must be >= 0");
    if (!(p->eps_reg > 0.f)) return fail(h, BODEX_EINVAL, "eps_reg must be positive");
    if (!std::isfinite(p->torque_scale)) return fail(h, BODEX_EINVAL, "torque_scale must be finite");
    if (!(p->tol_rel > 0.f)) return fail(h, BODEX_EINVAL, "tol_rel must be positive");
    if (p->max_iters < 1) return fail(h, BODEX_EINVAL, "max_iters must be >= 1");
    if (!(p->rho0 > 0.f)) return fail(h, BODEX_EINVAL, "rho0 must be positive");
    if (!(p->alpha > 0.f && p->alpha < 2.f)) return fail(h, BODEX_EINVAL, "alpha must be in (0, 2)");
    if (p->check_every < 1) return fail(h, BODEX_EINVAL, "check_every must be >= 1");
    if (!(p->rho_min > 0.f) || !(p->rho_max >= p->rho_min))
        return fail(h, BODEX_EINVAL, "need 0 < rho_min <= rho_max");
    if (p->polish_chunk < -1) return fail(h, BODEX_EINVAL, "polish_chunk must be >= -1");
    if (!(p->rho_hysteresis >= 1.f)) return fail(h, BODEX_EINVAL, "rho_hysteresis must be >= 1");
    if (!(p->fp64_cond > 0.f)) return fail(h, BODEX_EINVAL, "fp64_cond must be positive");
    if (p->polish_steps < 0) return fail(h, BODEX_EINVAL, "polish_steps must be >= 0");
    if (p->admm_waves < 0 || p->admm_waves > 4) return fail(h, BODEX_EINVAL, "admm_waves must be in [0, 4]");
    if (!(p->admm_tol >= 0.f)) return fail(h, BODEX_EINVAL, "admm_tol must be >= 0");
    if (p->friction_cone != BODEX_CONE_PYRAMID8 && p->friction_cone != BODEX_CONE_CIRCULAR)
        return fail(h, BODEX_EINVAL, "friction_cone must be BODEX_CONE_PYRAMID8 or BODEX_CONE_CIRCULAR");
    return 0;
}

KArgs make_args(const bodex_qp* h, const bodex_batch* in) {
    const bodex_qp_params& p = h->prm;
    const Effective e = effective(p, in->n_qps);
    KArgs a;
    std::memset(&a, 0, sizeof(a));
    a.points = in->points;
    a.normals = in->normals;
    a.mu = in->mu;
    a.wrench = in->wrench_dir;
    a.W = in->n_qps;
    a.sW = in->n_qps;
    a.ms = p.m_max;
    a.kappa = p.torque_scale;
    a.beta = p.beta;
    a.eps = p.eps_reg;
    a.fmax = p.force_max;
    a.gamma = p.gamma;
    a.tol = p.tol_rel;
    a.admm_tol = e.admm_tol;
    a.rho0 = p.rho0;
    a.alpha = p.alpha;
    a.rho_min = p.rho_min;
    a.rho_max = p.rho_max;
    a.hyst = p.rho_hysteresis;
    a.fp64_cond = p.fp64_cond;
    a.max_iters = e.max_iters;
    a.check_every = e.check_every;
    a.warm = (p.flags & BODEX_F_WARM_START) ? 1 : 0;
    a.adaptive = (p.flags & BODEX_F_ADAPTIVE_RHO) ? 1 : 0;
    a.polish = (p.flags & BODEX_F_POLISH) ? 1 : 0;
    a.polish_steps = p.polish_steps;
    a.cone = p.friction_cone == BODEX_CONE_CIRCULAR ? 1 : 0;
    return a;
}

// Validate the batch (host arrays only).  Returns 0 or an error code.
int validate_batch(bodex_qp* h, const bodex_batch* in) {
    if (!in) return fail(h, BODEX_EINVAL, "batch is NULL");
    const int G = in->n_grasps;
    if (G < 0) return fail(h, BODEX_EINVAL, "n_grasps < 0");
    if (G == 0) return 0;
    if (!in->contact_count || !in->wrench_offset)
        return fail(h, BODEX_EINVAL, "contact_count / wrench_offset (host arrays) are NULL");
    if (!in->points || !in->normals || !in->mu || !in->wrench_dir)
        return fail(h, BODEX_EINVAL, "an input device pointer is NULL");
    if (!aligned4(in->points) || !aligned4(in->normals) || !aligned4(in->mu) || !aligned4(in->wrench_dir))
        return fail(h, BODEX_EINVAL, "input pointers must be 4-byte aligned");
    const int* c = in->contact_count;
    const int* wo = in->wrench_offset;
    if (wo[0] != 0) return fail(h, BODEX_EINVAL, "wrench_offset[0] must be 0");
    for (int g = 0; g < G; ++g) {
        if (c[g] < 1 || c[g] > h->prm.m_max)
            return fail(h, BODEX_EINVAL, "grasp %d: contact count %d outside [1, %d]", g, c[g], h->prm.m_max);
        const int s = wo[g + 1] - wo[g];
        if (s < 1) return fail(h, BODEX_EINVAL, "grasp %d: %d wrenches (need >= 1)", g, s);
        if (s > h->prm.s_max)
            return fail(h, BODEX_EUNSUP, "grasp %d: %d wrenches exceed s_max=%d", g, s, h->prm.s_max);
        if (double(h->prm.gamma) > double(c[g]) * double(h->prm.force_max))
            return fail(h, BODEX_EINFEAS, "grasp %d: gamma=%g > m*fmax=%g", g, double(h->prm.gamma),
                        double(c[g]) * double(h->prm.force_max));
    }
    if (wo[G] != in->n_qps) return fail(h, BODEX_EINVAL, "n_qps=%d != wrench_offset[G]=%d", in->n_qps, wo[G]);
    return 0;
}

// Descriptor ints: counts | woff | perm | tile_start | [qp_offset |
// grasp_offset: with a pooled state layout] | queue(4).
size_t desc_ints(int G, const Schedule& S, bool lay) {
    return size_t(G) + (G + 1) + G + (S.n_tiles + 1) + (lay ? 2 * size_t(G) : 0) + 4;
}

// Whether st asks for a pooled state layout, and its validation (host
// arrays, before any device work).
int state_layout(bodex_qp* h, const bodex_batch* in, const bodex_state* st, bool* lay) {
    *lay = false;
    if (!st) return 0;
    if (!st->qp_offset && !st->grasp_offset) return 0;
    if (!st->qp_offset || !st->grasp_offset)
        return fail(h, BODEX_EINVAL, "state qp_offset and grasp_offset must both be set or both NULL");
    if (st->stride < 1 || st->rho_len < 1)
        return fail(h, BODEX_EINVAL, "a pooled state needs stride >= 1 and rho_len >= 1");
    for (int g = 0; g < in->n_grasps; ++g) {
        const int s = in->wrench_offset[g + 1] - in->wrench_offset[g];
        const long q = st->qp_offset[g];
        if (q < 0 || q + s > st->stride)
            return fail(h, BODEX_EINVAL, "state qp_offset[%d] = %ld with %d QPs outside [0, %d)", g, q, s,
                        st->stride);
        if (st->grasp_offset[g] < 0 || st->grasp_offset[g] >= st->rho_len)
            return fail(h, BODEX_EINVAL, "state grasp_offset[%d] = %d outside [0, %d)", g, st->grasp_offset[g],
                        st->rho_len);
    }
    *lay = true;
    return 0;
}

// Upload the descriptor (desc_ints) to `dst` via the pinned staging buffer;
// st: the pooled state layout or NULL.  Returns 0 or an error.
int upload_desc(bodex_qp* h, const bodex_batch* in, const Schedule& S, int* dst, size_t* n_ints_out,
                const bodex_state* st = nullptr) {
    const int G = in->n_grasps;
    const size_t n = desc_ints(G, S, st != nullptr);
    if (h->desc_pending) {
        HIP_TRY(h, hipEventSynchronize(h->desc_ev));
        h->desc_pending = false;
    }
    if (h->h_desc_cap < n) {
        if (h->h_desc) HIP_TRY(h, hipHostFree(h->h_desc));
        h->h_desc = nullptr;
        HIP_TRY(h, hipHostMalloc(reinterpret_cast<void**>(&h->h_desc), n * sizeof(int), hipHostMallocDefault));
        h->h_desc_cap = n;
    }
    int* p = h->h_desc;
    std::memcpy(p, in->contact_count, sizeof(int) * G);
    std::memcpy(p + G, in->wrench_offset, sizeof(int) * (G + 1));
    std::memcpy(p + 2 * G + 1, S.perm.data(), sizeof(int) * G);
    std::memcpy(p + 3 * G + 1, S.tile_start.data(), sizeof(int) * (S.n_tiles + 1));
    if (st) {
        std::memcpy(p + 3 * G + 2 + S.n_tiles, st->qp_offset, sizeof(int) * G);
        std::memcpy(p + 4 * G + 2 + S.n_tiles, st->grasp_offset, sizeof(int) * G);
    }
    std::memset(p + n - 4, 0, sizeof(int) * 4);
    HIP_TRY(h, hipMemcpyAsync(dst, p, n * sizeof(int), hipMemcpyHostToDevice, h->stream));
    HIP_TRY(h, hipEventRecord(h->desc_ev, h->stream));
    h->desc_pending = true;
    *n_ints_out = n;
    return 0;
}

void bind_desc(KArgs& a, const int* d, int G, const Schedule& S, bool lay = false) {
    a.counts = d;
    a.woff = d + G;
    a.perm = d + 2 * G + 1;
    a.tile_start = d + 3 * G + 1;
    a.n_tiles = S.n_tiles;
    a.slots = S.slots;
    a.sq = lay ? d + 3 * G + 2 + S.n_tiles : nullptr;
    a.sg = lay ? a.sq + G : nullptr;
}

// Validate a hand batch (pointers only; device contents are not read).
int validate_hand(bodex_qp* h, const bodex_hand* in) {
    if (!in) return fail(h, BODEX_EINVAL, "hand is NULL");
    if (in->n_grasps < 0) return fail(h, BODEX_EINVAL, "n_grasps %d < 0", in->n_grasps);
    if (in->m < 1 || in->m > BODEX_MAX_CONTACTS)
        return fail(h, BODEX_EINVAL, "m %d outside 1..%d", in->m, BODEX_MAX_CONTACTS);
    if (in->n_grasps == 0) return 0;
    if (!in->tip_local || !in->semi_axes || !in->hand_rot || !in->hand_trans)
        return fail(h, BODEX_EINVAL, "a hand array is NULL");
    const void* all[] = {in->contact_count, in->tip_local, in->semi_axes, in->hand_rot, in->hand_trans};
    for (const void* p : all)
        if (!aligned4(p)) return fail(h, BODEX_EINVAL, "hand arrays must be 4-byte aligned");
    return 0;
}

bodex::HandArgs hand_args(const bodex_qp* h, const bodex_hand* in) {
    bodex::HandArgs a;
    std::memset(&a, 0, sizeof(a));
    a.signed_dist = (h->prm.flags & BODEX_F_SIGNED_DIST) ? 1 : 0;
    a.G = in->n_grasps;
    a.M = in->m;
    a.counts = in->contact_count;
    a.tip = in->tip_local;
    a.axes = in->semi_axes;
    a.rot = in->hand_rot;
    a.trans = in->hand_trans;
    return a;
}

int occupancy_grid(bodex_qp* h, int blocks_per_cu_cap, int n_tiles) {
    int g = h->n_cu * blocks_per_cu_cap;
    return std::max(1, std::min(g, n_tiles));
}

}  // namespace

extern "C" {

void bodex_qp_default_params(bodex_qp_params* p) {
    if (!p) return;
    p->m_max = 5;
    p->s_max = 32;
    p->force_max = 1.0f;
    p->gamma = 0.0f;
    p->beta = 1.0f;
    p->eps_reg = 1e-6f;
    p->torque_scale = 20.0f;
    p->tol_rel = 1e-5f;
    p->max_iters = 500;
    p->rho0 = 0.3f;
    p->alpha = 1.6f;
    p->check_every = 10;
    p->rho_min = 1e-4f;
    p->rho_max = 1e4f;
    p->rho_hysteresis = 5.0f;
    p->fp64_cond = 1e4f;
    p->polish_steps = 128;
    p->polish_chunk = kDefaultPolishChunk;
    p->flags = BODEX_F_POLISH | BODEX_F_ADAPTIVE_RHO;
    p->admm_waves = 0;
    p->admm_tol = 0.0f;
}

int bodex_qp_create(const bodex_qp_params* p, int device, void* hip_stream, size_t hbm_budget_bytes,
                    bodex_qp_t** out) {
    if (!out) return fail(nullptr, BODEX_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate_params(p, nullptr);
    if (rc) return rc;
    if (kernel_mm(p->m_max) == 0)
        return fail(nullptr, BODEX_EUNSUP, "m_max=%d exceeds the contact counts this library was built for",
                    p->m_max);
    if (p->friction_cone == BODEX_CONE_CIRCULAR && p->m_max > kConeMaxMM)
        return fail(nullptr, BODEX_EUNSUP, "the circular cone is built for m_max <= %d (got %d)", kConeMaxMM,
                    p->m_max);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0)
        return fail(nullptr, BODEX_ENODEV, "no HIP device available");
    if (device < 0 || device >= ndev)
        return fail(nullptr, BODEX_EINVAL, "device %d outside [0, %d)", device, ndev);
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) return fail(nullptr, BODEX_EHIP, "hipSetDevice: %s", hipGetErrorString(e));
    bodex_qp* h = new (std::nothrow) bodex_qp();
    if (!h) return fail(nullptr, BODEX_EINVAL, "out of host memory");
    h->prm = *p;
    h->device = device;
    h->stream = static_cast<hipStream_t>(hip_stream);
    h->budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t(4) << 30);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        h->n_cu = prop.multiProcessorCount;
    e = hipEventCreateWithFlags(&h->desc_ev, hipEventDisableTiming);
    if (e != hipSuccess) {
        delete h;
        return fail(nullptr, BODEX_EHIP, "hipEventCreate: %s", hipGetErrorString(e));
    }
    // the static scratch's address on this device (bodex_qp_solve_static)
    int* sp = nullptr;
    if (static_scratch(h, device, &sp) != 0) {
        g_create_error = h->err;
        (void)hipEventDestroy(h->desc_ev);
        delete h;
        return BODEX_EHIP;
    }
    *out = h;
    return 0;
}

int bodex_qp_set_stream(bodex_qp_t* h, void* hip_stream) {
    if (!h) return BODEX_EINVAL;
    h->stream = static_cast<hipStream_t>(hip_stream);
    return 0;
}

int bodex_qp_solve(bodex_qp_t* h, const bodex_batch* in, bodex_result* out) {
    if (!h) return BODEX_EINVAL;
    if (!out) return fail(h, BODEX_EINVAL, "result is NULL");
    int rc = validate_batch(h, in);
    if (rc) return rc;
    h->last_launches = 0;
    h->last_replays = 0;
    h->last_tiles = 0;
    const int G = in->n_grasps;
    if (G == 0) return 0;
    const int W = in->n_qps;
    if (!out->forces || !out->qp_obj || !out->energy || !out->kkt_rel || !out->iters || !out->status)
        return fail(h, BODEX_EINVAL, "an output pointer is NULL");
    const bodex_state& st = out->state;
    const bool have_state = st.x || st.z || st.y || st.rho;
    if (have_state && !(st.x && st.z && st.y && st.rho))
        return fail(h, BODEX_EINVAL, "state pointers must be all set or all NULL");
    if ((h->prm.flags & BODEX_F_WARM_START) && !have_state)
        return fail(h, BODEX_EINVAL, "warm start needs the caller's state");
    bool lay = false;
    rc = state_layout(h, in, &st, &lay);
    if (rc) return rc;
    if (lay && !have_state) return fail(h, BODEX_EINVAL, "a pooled state layout needs the state pointers");
    HIP_TRY(h, hipSetDevice(h->device));

    const int mm = kernel_mm(h->prm.m_max);
    const bool cone = h->prm.friction_cone == BODEX_CONE_CIRCULAR;
    const int nv = 3 * h->prm.m_max, nr = (cone ? 3 : 9) * h->prm.m_max + 1;
    const bool batched = (h->prm.flags & BODEX_F_BATCHED) != 0;
    Schedule S;
    build_schedule(in->contact_count, in->wrench_offset, G, batched, S);
    h->last_tiles = S.n_tiles;

    KArgs a = make_args(h, in);
    if (have_state) {
        a.x = st.x;
        a.z = st.z;
        a.y = st.y;
        a.rho = st.rho;
        a.resid = st.r;
        if (lay) a.sW = st.stride;
    } else {
        const size_t need = (size_t(W) * (nv + 2 * nr) + size_t(G)) * sizeof(float);
        rc = ensure_device(h, reinterpret_cast<void**>(&h->d_state), &h->d_state_cap, need);
        if (rc) return rc;
        a.x = h->d_state;
        a.z = a.x + size_t(W) * nv;
        a.y = a.z + size_t(W) * nr;
        a.rho = a.y + size_t(W) * nr;
    }
    a.forces = out->forces;
    a.qobj = out->qp_obj;
    a.energy = out->energy;
    a.kkt = out->kkt_rel;
    a.iters = out->iters;
    a.status = out->status;
    a.pflops = out->polish_flops;

    bool chunked = false;
    int grid_g = 0;
    rc = chunk_setup(h, a, W, mm, chunked, grid_g);
    if (rc) return rc;

    const size_t n_ints = desc_ints(G, S, lay);
    const bool timing = (h->prm.flags & BODEX_F_TIMING) != 0;
    const bool graph = (h->prm.flags & BODEX_F_GRAPH) != 0 && h->stream != nullptr;
    const size_t lds_a = admm_lds(mm, S.slots);
    const size_t lds_f = cone ? bodex::cone_fin_lds(mm, S.slots, h->prm.gamma > 0.f) : fin_lds(mm, S.slots, false);
    int per_cu = std::max(1, std::min(16, int((160 * 1024) / std::max<size_t>(lds_a, 1))));
    const int grid_a = batched ? occupancy_grid(h, per_cu, S.n_tiles) : S.n_tiles;
    // finalize: one block per tile (the polish keeps its state in registers)
    const int grid_f = S.n_tiles;

    // Enqueue the launch sequence (reset counters, ADMM, finalize) for the
    // descriptors at d.
    auto enqueue = [&](int* d, bool with_events) -> int {
        bind_desc(a, d, G, S, lay);
        int* d_queue = d + (n_ints - 4);
        HIP_TRY(h, bodex::launch_reset(d_queue, 4, h->stream));
        KArgs aa = a;
        aa.queue = batched ? d_queue : nullptr;
        if (with_events) HIP_TRY(h, hipEventRecord(h->tev[0], h->stream));
        HIP_TRY(h, launch(Kind::Admm, mm, aa, grid_a, lds_a, h->stream, h->prm.admm_waves));
        if (with_events) HIP_TRY(h, hipEventRecord(h->tev[1], h->stream));
        KArgs f = a;
        f.queue = nullptr;
        if (with_events) HIP_TRY(h, hipEventRecord(h->tev[2], h->stream));
        rc = enqueue_finalize(h, f, mm, chunked, d_queue, grid_f, grid_g, lds_f);
        if (rc) return rc;
        if (with_events) HIP_TRY(h, hipEventRecord(h->tev[3], h->stream));
        return 0;
    };

    if (timing && !h->tev[0]) {
        for (auto& e : h->tev) HIP_TRY(h, hipEventCreate(&e));
    }
    h->t_admm = h->t_fin = false;

    if (!graph) {
        rc = ensure_device(h, reinterpret_cast<void**>(&h->d_desc), &h->d_desc_cap, n_ints * sizeof(int));
        if (rc) return rc;
        size_t up = 0;
        rc = upload_desc(h, in, S, h->d_desc, &up, lay ? &st : nullptr);
        if (rc) return rc;
        rc = enqueue(h->d_desc, timing);
        if (rc) return rc;
        h->last_launches = chunked ? 5 : 3;
        h->t_admm = h->t_fin = timing;
        return 0;
    }

    // Graph path: key on everything the captured launches depend on.
    uint64_t key = 1469598103934665603ull;
    key = fnv1a(key, &G, sizeof(G));
    key = fnv1a(key, in->contact_count, sizeof(int) * G);
    key = fnv1a(key, in->wrench_offset, sizeof(int) * (G + 1));
    if (lay) {
        key = fnv1a(key, st.qp_offset, sizeof(int) * G);
        key = fnv1a(key, st.grasp_offset, sizeof(int) * G);
    }
    key = fnv1a(key, &a, sizeof(a));
    key = fnv1a(key, &h->prm, sizeof(h->prm));
    GraphEntry* hit = nullptr;
    rc = graph_entry(h, key, n_ints, &hit);
    if (rc) return rc;
    if (!hit->exec) {
        size_t up = 0;
        rc = upload_desc(h, in, S, hit->d_desc, &up, lay ? &st : nullptr);
        if (rc) return rc;
        hipGraph_t gr = nullptr;
        HIP_TRY(h, hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
        rc = enqueue(hit->d_desc, false);
        hipError_t ce = hipStreamEndCapture(h->stream, &gr);
        if (rc) return rc;
        if (ce != hipSuccess) return hip_fail(h, ce, "hipStreamEndCapture");
        ce = hipGraphInstantiate(&hit->exec, gr, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gr);
        if (ce != hipSuccess) return hip_fail(h, ce, "hipGraphInstantiate");
    } else {
        h->last_replays = 1;
    }
    hit->stamp = ++h->graph_clock;
    if (timing) HIP_TRY(h, hipEventRecord(h->tev[0], h->stream));
    HIP_TRY(h, hipGraphLaunch(hit->exec, h->stream));
    if (timing) HIP_TRY(h, hipEventRecord(h->tev[1], h->stream));
    h->t_admm = timing;
    h->last_launches = 1;
    return 0;
}

int bodex_qp_solve_static(bodex_qp_t* h, const bodex_batch* in, bodex_result* out) {
    if (!h) return BODEX_EINVAL;
    int rc = validate_batch(h, in);
    if (rc) return rc;
    h->last_launches = 0;
    h->last_replays = 0;
    h->last_tiles = 0;
    if (h->prm.flags & (BODEX_F_BATCHED | BODEX_F_GRAPH))
        return fail(h, BODEX_EUNSUP, "bodex_qp_solve_static runs the plain form only (no BATCHED or GRAPH flag)");
    const int G = in->n_grasps;
    if (G == 0) return 0;
    if (!out->forces || !out->qp_obj || !out->energy || !out->kkt_rel || !out->iters || !out->status)
        return fail(h, BODEX_EINVAL, "an output pointer is NULL");
    const bodex_state& st = out->state;
    if (!(st.x && st.z && st.y && st.rho))
        return fail(h, BODEX_EINVAL, "bodex_qp_solve_static needs the caller's state (x, z, y, rho)");
    if (st.qp_offset || st.grasp_offset)
        return fail(h, BODEX_EUNSUP, "bodex_qp_solve_static takes the plain state layout only");
    // the plain schedule (consecutive grasps, at most kWave QPs and
    // kMaxSlots grasps per tile), built straight into the staging buffer
    const int* counts = in->contact_count;
    const int* woff = in->wrench_offset;
    int n_tiles = 0, slots = 1, cur_q = 0, cur_n = 0;
    for (int g = 0; g < G; ++g) {
        const int sg = woff[g + 1] - woff[g];
        if (cur_n > 0 && (cur_q + sg > bodex::kWave || cur_n >= bodex::kMaxSlots)) {
            ++n_tiles;
            slots = std::max(slots, cur_n);
            cur_q = cur_n = 0;
        }
        cur_q += sg;
        ++cur_n;
    }
    ++n_tiles;
    slots = std::max(slots, cur_n);
    const size_t n_ints = size_t(G) * 3 + 1 + size_t(n_tiles) + 1 + 4;
    if (n_ints > size_t(BODEX_STATIC_SCRATCH_INTS))
        return fail(h, BODEX_EUNSUP,
                    "batch needs %zu descriptor ints, beyond the static scratch of %d (every batch of up to %d "
                    "grasps fits)", n_ints, BODEX_STATIC_SCRATCH_INTS, (BODEX_STATIC_SCRATCH_INTS - 6) / 4);
    HIP_TRY(h, hipSetDevice(h->device));
    int* d = nullptr;
    rc = static_scratch(h, h->device, &d);
    if (rc) return rc;

    std::lock_guard<std::mutex> lk(g_static_mu);
    int* p = g_static_host;
    std::memcpy(p, counts, sizeof(int) * G);
    std::memcpy(p + G, woff, sizeof(int) * (G + 1));
    int* perm = p + 2 * G + 1;
    int* ts = p + 3 * G + 1;
    for (int g = 0; g < G; ++g) perm[g] = g;
    int t = 0;
    ts[0] = 0;
    cur_q = cur_n = 0;
    for (int g = 0; g < G; ++g) {
        const int sg = woff[g + 1] - woff[g];
        if (cur_n > 0 && (cur_q + sg > bodex::kWave || cur_n >= bodex::kMaxSlots)) {
            ts[++t] = g;
            cur_q = cur_n = 0;
        }
        cur_q += sg;
        ++cur_n;
    }
    ts[n_tiles] = G;
    std::memset(ts + n_tiles + 1, 0, sizeof(int) * 4);
    // pageable source: the copy has consumed the staging buffer when it returns
    HIP_TRY(h, hipMemcpyAsync(d, p, n_ints * sizeof(int), hipMemcpyHostToDevice, h->stream));

    const int mm = kernel_mm(h->prm.m_max);
    const bool cone = h->prm.friction_cone == BODEX_CONE_CIRCULAR;
    KArgs a = make_args(h, in);
    a.x = st.x;
    a.z = st.z;
    a.y = st.y;
    a.rho = st.rho;
    a.resid = st.r;
    a.forces = out->forces;
    a.qobj = out->qp_obj;
    a.energy = out->energy;
    a.kkt = out->kkt_rel;
    a.iters = out->iters;
    a.status = out->status;
    a.pflops = out->polish_flops;
    a.counts = d;
    a.woff = d + G;
    a.perm = d + 2 * G + 1;
    a.tile_start = d + 3 * G + 1;
    a.n_tiles = n_tiles;
    a.slots = slots;
    a.queue = nullptr;
    const size_t lds_a = admm_lds(mm, slots);
    const size_t lds_f = cone ? bodex::cone_fin_lds(mm, slots, h->prm.gamma > 0.f) : fin_lds(mm, slots, false);
    HIP_TRY(h, launch(Kind::Admm, mm, a, n_tiles, lds_a, h->stream, h->prm.admm_waves));
    HIP_TRY(h, launch(Kind::Fin, mm, a, n_tiles, lds_f, h->stream));
    h->last_launches = 2;
    h->last_tiles = n_tiles;
    return 0;
}

int bodex_qp_backward(bodex_qp_t* h, const bodex_batch* in, const bodex_state* st, const float* dL_dE,
                      const float* dL_dQ, float* dL_dpoints, float* dL_dnormals, int accumulate) {
    if (!h) return BODEX_EINVAL;
    int rc = validate_batch(h, in);
    if (rc) return rc;
    const int G = in->n_grasps;
    if (G == 0) return 0;
    if (!st || !st->x || !st->z || !st->y)
        return fail(h, BODEX_EINVAL, "backward needs the state written by a solve");
    if (!dL_dpoints || !dL_dnormals) return fail(h, BODEX_EINVAL, "gradient outputs are NULL");
    bool lay = false;
    rc = state_layout(h, in, st, &lay);
    if (rc) return rc;
    HIP_TRY(h, hipSetDevice(h->device));
    const int mm = kernel_mm(h->prm.m_max);
    Schedule S;
    build_schedule(in->contact_count, in->wrench_offset, G, false, S);
    KArgs a = make_args(h, in);
    a.x = st->x;
    a.z = st->z;
    a.y = st->y;
    a.rho = st->rho;
    a.resid = st->r;
    if (lay) a.sW = st->stride;
    a.dLdE = dL_dE;
    a.dLdQ = dL_dQ;
    a.dP = dL_dpoints;
    a.dN = dL_dnormals;
    a.accumulate = accumulate ? 1 : 0;
    const size_t n_ints = desc_ints(G, S, lay);
    rc = ensure_device(h, reinterpret_cast<void**>(&h->d_desc), &h->d_desc_cap, n_ints * sizeof(int));
    if (rc) return rc;
    size_t up = 0;
    rc = upload_desc(h, in, S, h->d_desc, &up, lay ? st : nullptr);
    if (rc) return rc;
    bind_desc(a, h->d_desc, G, S, lay);
    const size_t lds_b = fin_lds(mm, S.slots, true);
    a.queue = nullptr;
    const int grid_b = S.n_tiles;
    const bool timing = (h->prm.flags & BODEX_F_TIMING) != 0;
    if (timing && !h->tev[0]) {
        for (auto& e : h->tev) HIP_TRY(h, hipEventCreate(&e));
    }
    if (timing) HIP_TRY(h, hipEventRecord(h->tev[4], h->stream));
    HIP_TRY(h, launch(Kind::Bwd, mm, a, grid_b, lds_b, h->stream));
    if (timing) HIP_TRY(h, hipEventRecord(h->tev[5], h->stream));
    h->t_bwd = timing;
    h->last_launches = 2;
    return 0;
}

int bodex_qp_destroy(bodex_qp_t* h) {
    if (!h) return 0;
    (void)hipSetDevice(h->device);
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    else (void)hipDeviceSynchronize();
    for (auto& g : h->graphs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.d_desc) (void)hipFree(g.d_desc);
    }
    if (h->d_desc) (void)hipFree(h->d_desc);
    if (h->d_state) (void)hipFree(h->d_state);
    if (h->d_hand) (void)hipFree(h->d_hand);
    if (h->d_spill) (void)hipFree(h->d_spill);
    if (h->h_desc) (void)hipHostFree(h->h_desc);
    if (h->desc_ev) (void)hipEventDestroy(h->desc_ev);
    for (auto& e : h->tev)
        if (e) (void)hipEventDestroy(e);
    delete h;
    return 0;
}

const char* bodex_qp_last_error(const bodex_qp_t* h) {
    return h ? h->err.c_str() : g_create_error.c_str();
}

size_t bodex_qp_state_bytes(int n_grasps, int n_qps, int m_max) {
    if (n_grasps < 0 || n_qps < 0 || m_max < 1) return 0;
    const size_t nv = 3 * size_t(m_max), nr = 9 * size_t(m_max) + 1;
    return (size_t(n_qps) * (nv + 2 * nr + 6) + size_t(n_grasps)) * sizeof(float);
}

int bodex_qp_kernel_times(bodex_qp_t* h, float* admm_ms, float* finalize_ms, float* backward_ms) {
    if (!h) return BODEX_EINVAL;
    auto span = [&](bool valid, int i0, float* out) -> int {
        if (!out) return 0;
        *out = -1.f;
        if (!valid) return 0;
        HIP_TRY(h, hipEventSynchronize(h->tev[i0 + 1]));
        HIP_TRY(h, hipEventElapsedTime(out, h->tev[i0], h->tev[i0 + 1]));
        return 0;
    };
    int rc = span(h->t_admm, 0, admm_ms);
    if (!rc) rc = span(h->t_fin, 2, finalize_ms);
    if (!rc) rc = span(h->t_bwd, 4, backward_ms);
    return rc;
}

int bodex_qp_effective_params(const bodex_qp_params* p, int n_qps, float* admm_tol, int* max_iters,
                               int* check_every, int* polish_chunk) {
    if (!p || n_qps < 0) return fail(nullptr, BODEX_EINVAL, "params is NULL or n_qps < 0");
    const int rc = validate_params(p, nullptr);
    if (rc) return rc;
    const Effective e = effective(*p, n_qps);
    if (admm_tol) *admm_tol = e.admm_tol;
    if (max_iters) *max_iters = e.max_iters;
    if (check_every) *check_every = e.check_every;
    if (polish_chunk) *polish_chunk = e.polish_chunk;
    return 0;
}

int bodex_qp_last_stats(bodex_qp_t* h, int* launches, int* graph_replays, int* tiles) {
    if (!h) return BODEX_EINVAL;
    if (launches) *launches = h->last_launches;
    if (graph_replays) *graph_replays = h->last_replays;
    if (tiles) *tiles = h->last_tiles;
    return 0;
}

int bodex_qp_contact_query(bodex_qp_t* h, const bodex_hand* in, float* points, float* normals, float* dist) {
    if (!h) return BODEX_EINVAL;
    int rc = validate_hand(h, in);
    if (rc) return rc;
    if (in->n_grasps == 0) return 0;
    if (!points || !normals) return fail(h, BODEX_EINVAL, "points / normals are NULL");
    if (!aligned4(points) || !aligned4(normals) || !aligned4(dist))
        return fail(h, BODEX_EINVAL, "outputs must be 4-byte aligned");
    HIP_TRY(h, hipSetDevice(h->device));
    bodex::HandArgs a = hand_args(h, in);
    a.points = points;
    a.normals = normals;
    a.dist = dist;
    HIP_TRY(h, bodex::launch_hand_query(a, h->stream));
    h->last_launches = 1;
    return 0;
}

int bodex_qp_pose_gradient(bodex_qp_t* h, const bodex_hand* in, const float* dL_dpoints, const float* dL_dnormals,
                           float w_dist, float radius, float offset, float* e_dist, float* dL_drot,
                           float* dL_dtrans) {
    if (!h) return BODEX_EINVAL;
    int rc = validate_hand(h, in);
    if (rc) return rc;
    if (!std::isfinite(w_dist) || !std::isfinite(radius) || !std::isfinite(offset))
        return fail(h, BODEX_EINVAL, "w_dist, radius and offset must be finite");
    if (in->n_grasps == 0) return 0;
    const void* all[] = {dL_dpoints, dL_dnormals, e_dist, dL_drot, dL_dtrans};
    for (const void* p : all)
        if (!aligned4(p)) return fail(h, BODEX_EINVAL, "arrays must be 4-byte aligned");
    HIP_TRY(h, hipSetDevice(h->device));
    bodex::HandArgs a = hand_args(h, in);
    a.dLdp = dL_dpoints;
    a.dLdn = dL_dnormals;
    a.w_dist = w_dist;
    a.radius = radius;
    a.offset = offset;
    a.e_dist = e_dist;
    a.dLdrot = dL_drot;
    a.dLdtrans = dL_dtrans;
    HIP_TRY(h, bodex::launch_hand_step(a, h->stream));
    h->last_launches = 1;
    return 0;
}

int bodex_qp_descend(bodex_qp_t* h, const bodex_hand* hand, const bodex_batch* qp, const bodex_descent* d,
                     bodex_result* out, float* loss_trace) {
    if (!h) return BODEX_EINVAL;
    int rc = validate_hand(h, hand);
    if (rc) return rc;
    if (!qp || !d || !out) return fail(h, BODEX_EINVAL, "qp batch, descent parameters or result is NULL");
    if (hand->contact_count) return fail(h, BODEX_EINVAL, "hand->contact_count must be NULL (qp->contact_count is used)");
    if (qp->points || qp->normals) return fail(h, BODEX_EINVAL, "qp->points and qp->normals must be NULL");
    if (hand->m != h->prm.m_max) return fail(h, BODEX_EINVAL, "hand->m %d != m_max %d", hand->m, h->prm.m_max);
    if (qp->n_grasps != hand->n_grasps)
        return fail(h, BODEX_EINVAL, "qp->n_grasps %d != hand->n_grasps %d", qp->n_grasps, hand->n_grasps);
    if (d->iters < 0) return fail(h, BODEX_EINVAL, "iters %d < 0", d->iters);
    if (out->state.qp_offset || out->state.grasp_offset)
        return fail(h, BODEX_EUNSUP, "bodex_qp_descend takes the plain state layout only");
    const float fp[] = {d->w_qp, d->w_dist, d->radius, d->offset, d->step_rot, d->step_trans};
    for (float v : fp)
        if (!std::isfinite(v)) return fail(h, BODEX_EINVAL, "descent parameters must be finite");
    if (!aligned4(loss_trace)) return fail(h, BODEX_EINVAL, "loss_trace must be 4-byte aligned");
    const int G = hand->n_grasps, M = hand->m;
    h->last_launches = 0;
    if (G == 0 || d->iters == 0) return 0;
    if (!out->forces || !out->qp_obj || !out->energy || !out->kkt_rel || !out->iters || !out->status)
        return fail(h, BODEX_EINVAL, "an output pointer is NULL");
    const bodex_state& st = out->state;
    const bool have_state = st.x || st.z || st.y || st.rho;
    if (have_state && !(st.x && st.z && st.y && st.rho))
        return fail(h, BODEX_EINVAL, "state pointers must be all set or all NULL");
    if ((h->prm.flags & BODEX_F_WARM_START) && !have_state)
        return fail(h, BODEX_EINVAL, "warm start needs the caller's state");
    HIP_TRY(h, hipSetDevice(h->device));

    // workspace: points, normals, dL/dpoints, dL/dnormals [G][M][3], dist [G][M], w_qp [G]
    const size_t gm = size_t(G) * M;
    rc = ensure_device(h, reinterpret_cast<void**>(&h->d_hand), &h->d_hand_cap, (12 * gm + gm + G) * sizeof(float));
    if (rc) return rc;
    float* P = h->d_hand;
    float* N = P + 3 * gm;
    float* dP = N + 3 * gm;
    float* dN = dP + 3 * gm;
    float* D = dN + 3 * gm;
    float* wq = D + gm;
    bodex_batch qb = *qp;
    qb.points = P;
    qb.normals = N;
    rc = validate_batch(h, &qb);
    if (rc) return rc;
    const int W = qb.n_qps;

    const int mm = kernel_mm(h->prm.m_max);
    const bool cone = h->prm.friction_cone == BODEX_CONE_CIRCULAR;
    const int nv = 3 * h->prm.m_max, nr = (cone ? 3 : 9) * h->prm.m_max + 1;
    const bool batched = (h->prm.flags & BODEX_F_BATCHED) != 0;
    Schedule S;
    build_schedule(qb.contact_count, qb.wrench_offset, G, batched, S);
    h->last_tiles = S.n_tiles;
    KArgs a = make_args(h, &qb);
    if (have_state) {
        a.x = st.x;
        a.z = st.z;
        a.y = st.y;
        a.rho = st.rho;
        a.resid = st.r;
    } else {
        // the library's state, with the residual the backward of each step uses
        const size_t need = (size_t(W) * (nv + 2 * nr + 6) + size_t(G)) * sizeof(float);
        rc = ensure_device(h, reinterpret_cast<void**>(&h->d_state), &h->d_state_cap, need);
        if (rc) return rc;
        a.x = h->d_state;
        a.z = a.x + size_t(W) * nv;
        a.y = a.z + size_t(W) * nr;
        a.rho = a.y + size_t(W) * nr;
        a.resid = a.rho + size_t(G);
    }
    a.forces = out->forces;
    a.qobj = out->qp_obj;
    a.energy = out->energy;
    a.kkt = out->kkt_rel;
    a.iters = out->iters;
    a.status = out->status;
    a.pflops = out->polish_flops;
    const size_t n_ints = desc_ints(G, S, false);
    const size_t lds_a = admm_lds(mm, S.slots);
    const size_t lds_f = cone ? bodex::cone_fin_lds(mm, S.slots, h->prm.gamma > 0.f) : fin_lds(mm, S.slots, false);
    const size_t lds_b = fin_lds(mm, S.slots, true);
    const int per_cu = std::max(1, std::min(16, int((160 * 1024) / std::max<size_t>(lds_a, 1))));
    const int grid_a = batched ? occupancy_grid(h, per_cu, S.n_tiles) : S.n_tiles;
    bool chunked = false;
    int grid_g = 0;
    rc = chunk_setup(h, a, W, mm, chunked, grid_g);
    if (rc) return rc;

    // The whole descent for the descriptors at `desc`: loss weights, the
    // first contacts, then per step reset, ADMM, finalize, backward and the
    // pose step (which re-queries the contacts of the new pose).
    auto enqueue = [&](int* desc) -> int {
        KArgs ad = a;
        bind_desc(ad, desc, G, S);
        int* d_queue = desc + (n_ints - 4);
        bodex::HandArgs ha = hand_args(h, hand);
        ha.counts = ad.counts;  // the uploaded copy of qp->contact_count
        ha.points = P;
        ha.normals = N;
        ha.dist = D;
        HIP_TRY(h, bodex::launch_fill(wq, G, d->w_qp, h->stream));
        HIP_TRY(h, bodex::launch_hand_query(ha, h->stream));
        for (int k = 0; k < d->iters; ++k) {
            KArgs ak = ad;
            if (k > 0) ak.warm = 1;
            HIP_TRY(h, bodex::launch_reset(d_queue, 4, h->stream));
            ak.queue = batched ? d_queue : nullptr;
            HIP_TRY(h, launch(Kind::Admm, mm, ak, grid_a, lds_a, h->stream, h->prm.admm_waves));
            const int rf = enqueue_finalize(h, ak, mm, chunked, d_queue, S.n_tiles, grid_g, lds_f);
            if (rf) return rf;
            KArgs ab = ad;
            ab.queue = nullptr;
            ab.dLdE = wq;
            ab.dLdQ = nullptr;
            ab.dP = dP;
            ab.dN = dN;
            ab.accumulate = 0;
            HIP_TRY(h, launch(Kind::Bwd, mm, ab, S.n_tiles, lds_b, h->stream));
            bodex::HandArgs hs = ha;
            hs.dLdp = dP;
            hs.dLdn = dN;
            hs.e_qp = out->energy;
            hs.w_qp = d->w_qp;
            hs.w_dist = d->w_dist;
            hs.radius = d->radius;
            hs.offset = d->offset;
            hs.trace = loss_trace ? loss_trace + size_t(k) * G : nullptr;
            hs.step = 1;
            hs.step_rot = d->step_rot;
            hs.step_trans = d->step_trans;
            hs.requery = 1;
            HIP_TRY(h, bodex::launch_hand_step(hs, h->stream));
        }
        return 0;
    };

    const bool graph = (h->prm.flags & BODEX_F_GRAPH) != 0 && h->stream != nullptr;
    h->last_replays = 0;
    if (!graph) {
        rc = ensure_device(h, reinterpret_cast<void**>(&h->d_desc), &h->d_desc_cap, n_ints * sizeof(int));
        if (rc) return rc;
        size_t up = 0;
        rc = upload_desc(h, &qb, S, h->d_desc, &up);
        if (rc) return rc;
        rc = enqueue(h->d_desc);
        if (rc) return rc;
        h->last_launches = 2 + (chunked ? 7 : 5) * d->iters;
        return 0;
    }
    // Graph path: the descent's launches captured once per shape, pointers
    // and parameters, then replayed as one launch.
    uint64_t key = 0x9e3779b97f4a7c15ull;
    key = fnv1a(key, &G, sizeof(G));
    key = fnv1a(key, qb.contact_count, sizeof(int) * G);
    key = fnv1a(key, qb.wrench_offset, sizeof(int) * (G + 1));
    key = fnv1a(key, &a, sizeof(a));
    key = fnv1a(key, hand, sizeof(*hand));
    key = fnv1a(key, d, sizeof(*d));
    key = fnv1a(key, &loss_trace, sizeof(loss_trace));
    key = fnv1a(key, &h->d_hand, sizeof(h->d_hand));
    key = fnv1a(key, &h->prm, sizeof(h->prm));
    GraphEntry* hit = nullptr;
    rc = graph_entry(h, key, n_ints, &hit);
    if (rc) return rc;
    if (!hit->exec) {
        size_t up = 0;
        rc = upload_desc(h, &qb, S, hit->d_desc, &up);
        if (rc) return rc;
        hipGraph_t gr = nullptr;
        HIP_TRY(h, hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
        rc = enqueue(hit->d_desc);
        hipError_t ce = hipStreamEndCapture(h->stream, &gr);
        if (rc) return rc;
        if (ce != hipSuccess) return hip_fail(h, ce, "hipStreamEndCapture");
        ce = hipGraphInstantiate(&hit->exec, gr, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gr);
        if (ce != hipSuccess) return hip_fail(h, ce, "hipGraphInstantiate");
    } else {
        h->last_replays = 1;
    }
    hit->stamp = ++h->graph_clock;
    HIP_TRY(h, hipGraphLaunch(hit->exec, h->stream));
    h->last_launches = 1;
    return 0;
}

int bodex_qp_detach_energy(bodex_qp_t* h, const bodex_fine_contacts* in, const float* w_q, const float* w_e,
                           float* q_surr, float* e_dist, float* dL_dR, float* dL_dT, int accumulate) {
    if (!h) return BODEX_EINVAL;
    if (!in) return fail(h, BODEX_EINVAL, "fine contacts are NULL");
    const int G = in->n_grasps, M = in->m;
    if (G < 0) return fail(h, BODEX_EINVAL, "n_grasps %d < 0", G);
    if (M < 1 || M > BODEX_MAX_CONTACTS) return fail(h, BODEX_EINVAL, "m %d outside 1..%d", M, BODEX_MAX_CONTACTS);
    if ((dL_dR == nullptr) != (dL_dT == nullptr))
        return fail(h, BODEX_EINVAL, "dL_dR and dL_dT must both be set or both be NULL");
    if (G == 0) return 0;
    const void* req[] = {in->link_rot, in->link_trans, in->hand_fine, in->obj_fine, in->obj_coarse, q_surr, e_dist};
    for (const void* p : req)
        if (!p) return fail(h, BODEX_EINVAL, "a required array is NULL");
    const void* all[] = {in->contact_count, in->link_rot, in->link_trans, in->hand_fine, in->obj_fine,
                         in->obj_coarse, w_q, w_e, q_surr, e_dist, dL_dR, dL_dT};
    for (const void* p : all)
        if (!aligned4(p)) return fail(h, BODEX_EINVAL, "arrays must be 4-byte aligned");
    HIP_TRY(h, hipSetDevice(h->device));
    bodex::DetachArgs a;
    a.G = G;
    a.M = M;
    a.counts = in->contact_count;
    a.R = in->link_rot;
    a.T = in->link_trans;
    a.cw = in->hand_fine;
    a.pf = in->obj_fine;
    a.pc = in->obj_coarse;
    a.wq = w_q;
    a.we = w_e;
    a.Qp = q_surr;
    a.Ed = e_dist;
    a.dR = dL_dR;
    a.dT = dL_dT;
    a.accumulate = accumulate ? 1 : 0;
    HIP_TRY(h, bodex::launch_detach(a, h->stream));
    h->last_launches = 1;
    return 0;
}

}  // extern "C"
