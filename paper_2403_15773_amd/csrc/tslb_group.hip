// Serving: a group of lattices advanced together by one multi-domain fused
// step launch (continuous batching at step granularity).  Declarations and
// contracts are in include/tslb.h.
//
// Each tslb_group_poll() call retires the members whose last step has finished
// on the device and launches one step of every member with steps left.  A
// launch reads a device table of FusedDomain records (one per member, grouped
// by storage type); the tables live in a ring of kRing slots so that up to
// kRing launches are in flight, and a slot's pinned host copy is rewritten only
// after the event of the launch that last used it has completed.
#include <algorithm>
#include <functional>
#include <new>
#include <string>
#include <vector>

#include "tslb_internal.h"

using namespace tslb;

struct tslb_group {
    static constexpr int kRing = 4;
    size_t budget = 0;
    int max_domains = 0;
    int device = 0;
    hipStream_t stream = nullptr;
    bool owns_stream = false;
    size_t bytes_in_use = 0;
    struct Member {
        tslb_ctx *ctx;
        int64_t remaining;    // steps still to launch
        int64_t last_launch;  // launch that wrote its newest state (-1: none)
        size_t bytes;         // HBM charged against the budget
    };
    std::vector<Member> members;  // in admission order
    FusedDomain *h_tab[kRing] = {};
    FusedDomain *d_tab[kRing] = {};
    hipEvent_t ev[kRing] = {};     // end of launch (slot reuse and retirement)
    hipEvent_t ev_start[kRing] = {};  // start of launch (device-busy time)
    double busy_ms = 0.0;          // summed durations of the completed launches
    int64_t slot_launch[kRing] = {-1, -1, -1, -1};
    int64_t launches = 0;        // launches issued
    int64_t completed = -1;      // every launch <= completed has finished
    hipEvent_t admit_ev = nullptr;
    std::string err;
    // chunk bound of each launch class (storage type x {one component, two with
    // 16-row tiles, two with 20-row tiles}, and the variable-density step), kept
    // while the class's stepping members stay the same
    static constexpr int kPlanClasses = 3 * 4 + 1;
    std::vector<const tslb_ctx *> plan_members[kPlanClasses];
    int plan_bound[kPlanClasses] = {};
};

namespace {

constexpr int kStorageTypes = 4;  // TSLB_STORE_FP32 .. TSLB_STORE_FP16Q
// launch classes: storage type x {one component, two components on 16-row
// tiles, two on 20-row tiles}, plus the variable-density step (binary32, two
// components, 16 rows) as a class of its own
constexpr int kClasses = 3 * kStorageTypes + 1;
constexpr int kClassVD = 3 * kStorageTypes;
static_assert(kClasses == tslb_group::kPlanClasses, "one chunk plan per launch class");
int class_of(const tslb_ctx *c) {
    return c->vd ? kClassVD : 3 * c->storage + (c->phase ? (fused_rows(c) == 20 ? 2 : 1) : 0);
}

int gfail(tslb_group *g, int code, const std::string &msg) {
    if (g)
        g->err = msg;
    else
        set_thread_error(msg);
    return code;
}

#define GHIP_TRY(g, expr)                                                                                 \
    do {                                                                                                  \
        hipError_t e_ = (expr);                                                                           \
        if (e_ != hipSuccess)                                                                             \
            return gfail((g), TSLB_E_DEVICE, std::string(#expr) + " failed: " + hipGetErrorString(e_));   \
    } while (0)

// Advance g->completed over the launches whose slot events have fired.
int refresh_completed(tslb_group *g) {
    while (g->completed + 1 < g->launches) {
        const int64_t next = g->completed + 1;
        const int slot = (int)(next % tslb_group::kRing);
        const hipError_t q = hipEventQuery(g->ev[slot]);
        if (q == hipErrorNotReady) break;
        if (q != hipSuccess) return gfail(g, TSLB_E_DEVICE, std::string("hipEventQuery: ") + hipGetErrorString(q));
        float ms = 0.f;
        const hipError_t e = hipEventElapsedTime(&ms, g->ev_start[slot], g->ev[slot]);
        if (e != hipSuccess) return gfail(g, TSLB_E_DEVICE, std::string("hipEventElapsedTime: ") + hipGetErrorString(e));
        g->busy_ms += ms;
        g->completed = next;
    }
    return TSLB_OK;
}

// z chunk length of a lattice of nz planes under the bound L: ceil(nz / L)
// chunks of near-equal length.
int chunk_under_bound(int nz, int L) {
    const int k = (nz + L - 1) / L;
    return (nz + k - 1) / k;
}

// End time, in pipeline planes, of one launch whose work items take cost[i]
// planes each: the items are split into eight contiguous ranges, one per XCD
// (xcd_work_item), and the compute units of an XCD take their range's items
// in order as they free up.
long long launch_end(const std::vector<int> &cost, int cus, std::vector<long long> &heap) {
    const int n = (int)cost.size(), per_xcd = std::max(1, cus / 8);
    const int q8 = n >> 3, rem8 = n & 7;
    long long end = 0;
    int begin = 0;
    for (int x = 0; x < 8; ++x) {
        const int cnt = q8 + (x < rem8 ? 1 : 0);
        heap.assign((size_t)std::min(per_xcd, std::max(cnt, 1)), 0);  // free times, a min-heap
        for (int i = begin; i < begin + cnt; ++i) {
            std::pop_heap(heap.begin(), heap.end(), std::greater<long long>());
            heap.back() += cost[(size_t)i];
            std::push_heap(heap.begin(), heap.end(), std::greater<long long>());
        }
        for (long long t : heap) end = std::max(end, t);
        begin += cnt;
    }
    return end;
}

// The chunk bound of launch class cl: every stepping member of the class
// splits its z extent into chunks under one bound L, and the launch takes the
// L whose simulated end time is earliest (a workgroup on a chunk of l planes
// walks l + 6 pipeline planes, so long chunks recompute less, short ones leave
// fewer compute units idle while the last items finish).  The choice is kept
// until a member is admitted or leaves, or one of the class stops stepping.
// The result of a step does not depend on the chunk length.
int plan_chunk_bound(tslb_group *g, int cl) {
    std::vector<const tslb_ctx *> now;
    int cus = 0;
    for (const tslb_group::Member &m : g->members)
        if (m.remaining > 0 && class_of(m.ctx) == cl) {
            now.push_back(m.ctx);
            cus = std::max(cus, m.ctx->cu_count);
        }
    if (now.empty()) return 64;
    if (now == g->plan_members[cl] && g->plan_bound[cl] > 0) return g->plan_bound[cl];
    static const int kBounds[] = {8, 12, 16, 24, 32, 48, 64, 96, 128};
    std::vector<int> cost;
    std::vector<long long> heap;
    long long best = -1;
    int best_L = 64;
    for (int L : kBounds) {
        cost.clear();
        for (const tslb_ctx *c : now) {
            const int nz = c->geo.nz, lz = chunk_under_bound(nz, L);
            const int chunks = (nz + lz - 1) / lz;
            const int tiles = fused_work_items(c, nz);  // one chunk of nz planes: the tile count
            for (int j = 0; j < chunks; ++j) {
                const int planes = std::min(lz, nz - j * lz) + 6;
                for (int t = 0; t < tiles; ++t) cost.push_back(planes);
            }
        }
        const long long e = launch_end(cost, std::max(cus, 8), heap);
        if (best < 0 || e <= best) {  // ties go to the longer chunks
            best = e;
            best_L = L;
        }
    }
    g->plan_members[cl] = now;
    g->plan_bound[cl] = best_L;
    return best_L;
}

void release_all(tslb_group *g) {
    for (int s = 0; s < tslb_group::kRing; ++s) {
        if (g->ev[s]) (void)hipEventDestroy(g->ev[s]);
        if (g->ev_start[s]) (void)hipEventDestroy(g->ev_start[s]);
        if (g->d_tab[s]) (void)hipFree(g->d_tab[s]);
        if (g->h_tab[s]) (void)hipHostFree(g->h_tab[s]);
    }
    if (g->admit_ev) (void)hipEventDestroy(g->admit_ev);
    if (g->owns_stream && g->stream) (void)hipStreamDestroy(g->stream);
}

}  // namespace

namespace tslb {

// Remove ctx from its group (tslb_destroy of a member): wait for the group's
// work, then forget the member and return its bytes to the budget.
void group_detach(tslb_group *g, tslb_ctx *c) {
    if (!g || !c) return;
    (void)hipStreamSynchronize(g->stream);
    for (size_t i = 0; i < g->members.size(); ++i)
        if (g->members[i].ctx == c) {
            g->bytes_in_use -= g->members[i].bytes;
            g->members.erase(g->members.begin() + (long)i);
            break;
        }
    for (int &b : g->plan_bound) b = 0;  // a later context may reuse c's address
    c->group = nullptr;
}

}  // namespace tslb

extern "C" {

int tslb_group_create(size_t hbm_budget_bytes, int32_t max_domains, void *stream, tslb_group **out) {
    if (!out) return gfail(nullptr, TSLB_E_INVAL, "out is NULL");
    *out = nullptr;
    if (max_domains < 1 || max_domains > 4096) return gfail(nullptr, TSLB_E_INVAL, "max_domains must be in [1, 4096]");
    if (hbm_budget_bytes == 0) return gfail(nullptr, TSLB_E_INVAL, "hbm_budget_bytes must be positive");
    tslb_group *g = new (std::nothrow) tslb_group();
    if (!g) return gfail(nullptr, TSLB_E_NOMEM, "host allocation failed");
    g->budget = hbm_budget_bytes;
    g->max_domains = max_domains;
    hipError_t e = hipGetDevice(&g->device);
    // every member has one record per launch: max_domains records per slot
    const size_t tab = (size_t)max_domains * sizeof(FusedDomain);
    for (int s = 0; e == hipSuccess && s < tslb_group::kRing; ++s) {
        e = hipHostMalloc((void **)&g->h_tab[s], tab, hipHostMallocDefault);
        if (e == hipSuccess) e = hipMalloc((void **)&g->d_tab[s], tab);
        if (e == hipSuccess) e = hipEventCreate(&g->ev[s]);
        if (e == hipSuccess) e = hipEventCreate(&g->ev_start[s]);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&g->admit_ev, hipEventDisableTiming);
    if (e == hipSuccess) {
        if (stream) {
            g->stream = (hipStream_t)stream;
        } else {
            e = hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking);
            g->owns_stream = e == hipSuccess;
        }
    }
    if (e != hipSuccess) {
        const int code = e == hipErrorOutOfMemory ? TSLB_E_NOMEM : TSLB_E_DEVICE;
        release_all(g);
        delete g;
        return gfail(nullptr, code, std::string("group set-up failed: ") + hipGetErrorString(e));
    }
    *out = g;
    return TSLB_OK;
}

int tslb_group_admit(tslb_group *g, tslb_ctx *c, int64_t nsteps) {
    if (!g) return gfail(nullptr, TSLB_E_INVAL, "group is NULL");
    if (!c) return gfail(g, TSLB_E_INVAL, "ctx is NULL");
    if (nsteps < 0) return gfail(g, TSLB_E_INVAL, "nsteps must be >= 0");
    if (c->group) return gfail(g, TSLB_E_STATE, "ctx is already in a group");
    if (!c->state_set) return gfail(g, TSLB_E_STATE, "ctx has no state");
    if (c->kernel != TSLB_KERNEL_FUSED) return gfail(g, TSLB_E_STATE, "groups run the fused step kernel only");
    if (c->p.device != g->device) return gfail(g, TSLB_E_INVAL, "ctx and group are on different devices");
    if ((int)g->members.size() >= g->max_domains) return gfail(g, TSLB_E_NOMEM, "all domain slots are taken");
    GHIP_TRY(g, hipSetDevice(g->device));
    const size_t bytes = ctx_device_bytes(c);
    if (g->bytes_in_use + bytes > g->budget) return gfail(g, TSLB_E_NOMEM, "HBM budget exhausted");
    try {
        g->members.reserve(g->members.size() + 1);
    } catch (const std::bad_alloc &) {
        return gfail(g, TSLB_E_NOMEM, "host allocation failed");
    }
    // the group stream starts after everything already queued on the ctx
    GHIP_TRY(g, hipEventRecord(g->admit_ev, c->stream));
    GHIP_TRY(g, hipStreamWaitEvent(g->stream, g->admit_ev, 0));
    // the fused step writes the boundary layers of the states it produces; the
    // current state's layers are filled once here (the fill is idempotent)
    if (nsteps > 0) GHIP_TRY(g, launch_boundary(c, c->buf[c->cur], c->step, g->stream));
    // a member with no steps is done once the work queued so far has finished
    g->members.push_back({c, nsteps, nsteps > 0 ? -1 : g->launches - 1, bytes});  // reserved: no throw
    g->bytes_in_use += bytes;
    for (int &b : g->plan_bound) b = 0;
    c->group = g;
    return TSLB_OK;
}

int tslb_group_poll(tslb_group *g, tslb_ctx **done, int32_t cap, int32_t *ndone) {
    if (!g) return gfail(nullptr, TSLB_E_INVAL, "group is NULL");
    if (!ndone) return gfail(g, TSLB_E_INVAL, "ndone is NULL");
    if (cap < 0 || (cap > 0 && !done)) return gfail(g, TSLB_E_INVAL, "done/cap invalid");
    *ndone = 0;
    GHIP_TRY(g, hipSetDevice(g->device));
    int rc = refresh_completed(g);
    if (rc) return rc;
    // retire members whose newest state is complete (admission order)
    for (size_t i = 0; i < g->members.size() && *ndone < cap;) {
        tslb_group::Member &m = g->members[i];
        if (m.remaining == 0 && m.last_launch <= g->completed) {
            if (m.last_launch < 0) {  // no launch at all: wait for its boundary fill
                const hipError_t q = hipStreamQuery(g->stream);
                if (q == hipErrorNotReady) { ++i; continue; }
                if (q != hipSuccess) return gfail(g, TSLB_E_DEVICE, std::string("hipStreamQuery: ") + hipGetErrorString(q));
            }
            done[(*ndone)++] = m.ctx;
            m.ctx->group = nullptr;
            g->bytes_in_use -= m.bytes;
            g->members.erase(g->members.begin() + (long)i);
        } else {
            ++i;
        }
    }
    // one step of every member with steps left
    bool any = false;
    for (const tslb_group::Member &m : g->members) any = any || m.remaining > 0;
    if (!any) return TSLB_OK;
    const int64_t id = g->launches;
    const int slot = (int)(id % tslb_group::kRing);
    if (g->slot_launch[slot] >= 0 && g->slot_launch[slot] > g->completed) {
        GHIP_TRY(g, hipEventSynchronize(g->ev[slot]));
        rc = refresh_completed(g);
        if (rc) return rc;
    }
    FusedDomain *h = g->h_tab[slot];
    int nrec = 0;
    // one launch per class (storage type, component count, tile height; variable density) present
    int first[kClasses] = {}, count[kClasses] = {}, work[kClasses] = {};
    for (int cl = 0; cl < kClasses; ++cl) {
        first[cl] = nrec;
        const int bound = plan_chunk_bound(g, cl);
        for (tslb_group::Member &m : g->members) {
            tslb_ctx *c = m.ctx;
            if (m.remaining <= 0 || class_of(c) != cl) continue;
            h[nrec] = fused_domain(c, c->buf[c->cur], c->buf[c->cur ^ 1], c->step + 1, work[cl],
                                   chunk_under_bound(c->geo.nz, bound));
            work[cl] += h[nrec].work_count;
            ++nrec;
            ++count[cl];
        }
    }
    GHIP_TRY(g, hipEventRecord(g->ev_start[slot], g->stream));
    GHIP_TRY(g, hipMemcpyAsync(g->d_tab[slot], h, (size_t)nrec * sizeof(FusedDomain), hipMemcpyHostToDevice,
                               g->stream));
    for (int cl = 0; cl < kClasses; ++cl)
        if (count[cl])
            GHIP_TRY(g, launch_step_fused_multi(g->d_tab[slot] + first[cl], count[cl], work[cl],
                                                cl == kClassVD ? (int)ST_FP32 : cl / 3,
                                                cl == kClassVD || cl % 3 != 0, cl == kClassVD,
                                                cl != kClassVD && cl % 3 == 2 ? 20 : 16, g->stream));
    GHIP_TRY(g, hipEventRecord(g->ev[slot], g->stream));
    g->slot_launch[slot] = id;
    g->launches = id + 1;
    for (tslb_group::Member &m : g->members) {
        if (m.remaining <= 0) continue;
        m.ctx->cur ^= 1;
        m.ctx->step += 1;
        m.remaining -= 1;
        m.last_launch = id;
    }
    return TSLB_OK;
}

int tslb_group_status(const tslb_group *g, size_t *bytes_in_use, int32_t *members, int64_t *launches) {
    if (!g) return gfail(nullptr, TSLB_E_INVAL, "group is NULL");
    if (bytes_in_use) *bytes_in_use = g->bytes_in_use;
    if (members) *members = (int32_t)g->members.size();
    if (launches) *launches = g->launches;
    return TSLB_OK;
}

int tslb_group_busy(tslb_group *g, double *busy_ms, int64_t *completed) {
    if (!g) return gfail(nullptr, TSLB_E_INVAL, "group is NULL");
    GHIP_TRY(g, hipSetDevice(g->device));
    int rc = refresh_completed(g);
    if (rc) return rc;
    if (busy_ms) *busy_ms = g->busy_ms;
    if (completed) *completed = g->completed + 1;
    return TSLB_OK;
}

void tslb_group_destroy(tslb_group *g) {
    if (!g) return;
    (void)hipSetDevice(g->device);
    if (g->stream) (void)hipStreamSynchronize(g->stream);
    for (tslb_group::Member &m : g->members) m.ctx->group = nullptr;
    release_all(g);
    delete g;
}

const char *tslb_group_last_error(const tslb_group *g) { return g ? g->err.c_str() : tslb_last_error(nullptr); }

}  // extern "C"
