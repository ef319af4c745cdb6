// vkt_batch.hip -- vktApplyFilterBatched: many independent ApplyFilter calls
// of uneven volume sizes and mixed filter sizes in persistent launches.
//
// Planning (host, once per distinct batch):
//   * every (dst, src, filter) triple is validated and planned exactly as by
//     vktApplyFilter; triples fall into arithmetic classes (cell format, k,
//     vector-ALU or matrix-core path and its variant), one persistent kernel
//     per class;
//   * each volume is cut into tile-slabs (the kernel's output tile -- one of
//     two tile heights -- times a z-slab depth, both chosen per class and
//     batch size class, by default or by the autotuner, which times every
//     tile height at candidate depths on the real batch); the class's work
//     list is sorted longest first;
//   * descriptors, work lists, the classes' weight pools and the work-queue
//     counters go to one device buffer; the class kernels become parallel
//     kernel nodes of one hipGraph.
// Launch: one hipGraphLaunch on the calling thread's stream.  Plans are cached
// by the batch's signature (pointers, dims, formats, filter identities, mode,
// precision, stream), so repeated batches replay the instantiated graph.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "vkt_internal.h"

namespace vkt {
namespace {

struct ClassKey {
    // path 0 = vector ALU (flag: int accumulate), 1 = matrix (flag bit 0: 6
    // products, bit 1: row-pair kernel), 2 = 8-bit dot products (flag:
    // signed weights)
    int fmt, k, path, flag;
    bool operator<(const ClassKey& o) const
    {
        return std::tie(fmt, k, path, flag) < std::tie(o.fmt, o.k, o.path, o.flag);
    }
};

// variant: the class's tile-height variant (0: default tile, 1: the other
// height; kTileVariants in all)
const void* class_kernel(const ClassKey& c, int variant)
{
    if (c.path == 2) return dot4_batched_kernel(c.k, c.flag != 0, variant);
    return c.path ? mfma_batched_kernel((vktDataFormat)c.fmt, c.k, (c.flag & 1) != 0,
                                        (c.flag & 2) != 0, variant)
                  : valu_batched_kernel((vktDataFormat)c.fmt, c.k, c.flag != 0, variant);
}

ClassGeom class_geom(const ClassKey& c, int variant)
{
    if (c.path == 2) return dot4_geom(c.k, variant);
    return c.path ? mfma_geom((vktDataFormat)c.fmt, c.k, (c.flag & 1) != 0, (c.flag & 2) != 0,
                              variant)
                  : valu_geom(c.k, variant);
}

// Weights per filter in the class's pools: k^3 (float and int pools), or the
// packed 8-bit rows (int pool) of the dot-product path.
int class_weights(const ClassKey& c) { return c.path == 2 ? dot4_words(c.k) : c.k * c.k * c.k; }

// ---- tuning table: (class, size class) -> tile variant and z-slab depth ----

struct TuneKey {
    ClassKey c;
    int size_class;
    bool operator<(const TuneKey& o) const
    {
        return std::tie(c, size_class) < std::tie(o.c, o.size_class);
    }
};

struct TuneVal {
    int tz;        // z-slab depth (0: no entry)
    int variant;   // tile-height variant
};

std::mutex g_tune_mu;
std::map<TuneKey, TuneVal> g_tune;
bool g_tune_loaded = false;

// Size class of a set of volumes: log2 of the mean cube-root edge length.
int size_class_of(const std::vector<FilterJob>& jobs)
{
    double s = 0;
    for (const auto& j : jobs) s += std::cbrt((double)j.X * j.Y * j.Z);
    return jobs.empty() ? 0 : (int)std::floor(std::log2(s / (double)jobs.size()));
}

void tune_load_locked()
{
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char* path = std::getenv("VKT_TUNE_CACHE");
    if (!path) return;
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    char line[256];
    while (std::fgets(line, sizeof line, f)) {
        TuneKey k;
        TuneVal v{0, 0};
        // fmt k path flag size_class tz [variant]
        const int n = std::sscanf(line, "%d %d %d %d %d %d %d", &k.c.fmt, &k.c.k, &k.c.path,
                                  &k.c.flag, &k.size_class, &v.tz, &v.variant);
        if (n >= 6 && v.tz > 0 && v.variant >= 0 && v.variant < kTileVariants) g_tune[k] = v;
    }
    std::fclose(f);
}

void tune_store_locked()
{
    const char* path = std::getenv("VKT_TUNE_CACHE");
    if (!path) return;
    FILE* f = std::fopen(path, "w");
    if (!f) return;
    for (const auto& e : g_tune)
        std::fprintf(f, "%d %d %d %d %d %d %d\n", e.first.c.fmt, e.first.c.k, e.first.c.path,
                     e.first.c.flag, e.first.size_class, e.second.tz, e.second.variant);
    std::fclose(f);
}

int default_tz(const ClassKey& c, const ClassGeom& g)
{
    (void)c;
    return std::max(g.tz_min, 16);
}

// ---- plans ------------------------------------------------------------------

struct ClassPlan {
    ClassKey key;
    const void* func = nullptr;
    std::vector<int> members;      // indices into the batch
    int tz = 0;
    int variant = 0;               // tile-height variant
    unsigned grid = 0;
    BatchArgs args{};
    // offsets inside the plan's device buffer
    size_t off_desc = 0, off_items = 0, off_cnt = 0, off_wf = 0, off_wi = 0;
    uint32_t nitems = 0;
};

struct Plan {
    std::vector<uintptr_t> sig;
    int device = 0;
    char* dbuf = nullptr;
    size_t dbytes = 0;
    std::vector<ClassPlan> classes;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // recorded after every launch of the graph: an evicted plan is destroyed
    // only once its last launch has finished (the launch may still be queued
    // on another thread's stream when the plan leaves the cache)
    hipEvent_t done = nullptr;
    ~Plan()
    {
        if (done) {
            (void)hipEventSynchronize(done);
            (void)hipEventDestroy(done);
        }
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (dbuf) (void)hipFree(dbuf);
    }
};

// Plan cache, least recently used first.  Plans are shared: a caller holds
// its plan until its graph launch has been enqueued, so a plan evicted by
// another thread meanwhile stays alive until then (the graph itself may still
// be running when the last holder lets go; hipFree of the plan's buffer waits
// for it).
std::mutex g_plan_mu;
std::vector<std::shared_ptr<Plan>> g_plans;
constexpr size_t kMaxPlans = 16;

// Batched calls from several threads run one at a time inside the library:
// planning, graph instantiation, launch and the destruction of evicted plans
// are serialised (a two-thread test that fills the cache past its capacity
// crashed inside this call with them running concurrently; the library's own
// shared state is locked, so the HIP graph calls are the suspects).  The
// enqueued work itself still runs concurrently on the callers' streams.
std::mutex g_batch_mu;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Work list of one class at slab depth tz, longest items first.
std::vector<WorkItem> make_items(const std::vector<VolDesc>& descs,
                                 const std::vector<int>& members, int k)
{
    struct Costed {
        WorkItem w;
        int64_t cost;
    };
    std::vector<Costed> v;
    for (size_t m = 0; m < members.size(); ++m) {
        const VolDesc& a = descs[m];
        const int64_t nt = (int64_t)a.tiles_x * a.tiles_y;
        const int slabs = (a.Z + a.tz - 1) / a.tz;
        for (int sl = 0; sl < slabs; ++sl) {
            const int planes = std::min(a.tz, a.Z - sl * a.tz) + k - 1;
            for (int64_t t = 0; t < nt; ++t) {
                Costed c;
                c.w.vol = (uint32_t)m;
                c.w.lid = (uint32_t)(sl * nt + t);
                c.cost = planes;
                v.push_back(c);
            }
        }
    }
    std::stable_sort(v.begin(), v.end(),
                     [](const Costed& a, const Costed& b) { return a.cost > b.cost; });
    std::vector<WorkItem> out(v.size());
    for (size_t i = 0; i < v.size(); ++i) out[i] = v[i].w;
    return out;
}

struct Triple {
    FilterJob j;
    ClassKey key;
    const vktFilter_* f;
};

// Tuning-table key of one class of a batch, and the entry the table holds
// for it (tz 0: none).
TuneKey tune_key(const std::vector<Triple>& tr, const ClassPlan& cp)
{
    std::vector<FilterJob> jobs;
    for (int idx : cp.members) jobs.push_back(tr[idx].j);
    return TuneKey{cp.key, size_class_of(jobs)};
}

TuneVal tuned(const TuneKey& tk)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_locked();
    auto it = g_tune.find(tk);
    return it != g_tune.end() ? it->second : TuneVal{0, 0};
}

// Build (or rebuild for another slab depth) the host-side arrays of one class.
void class_arrays(const std::vector<Triple>& tr, ClassPlan& cp, std::vector<VolDesc>& descs,
                  std::vector<WorkItem>& items, std::vector<float>& wf,
                  std::vector<int32_t>& wi)
{
    const ClassGeom g = class_geom(cp.key, cp.variant);
    descs.clear();
    wf.clear();
    wi.clear();
    std::map<uint64_t, uint32_t> woff;  // filter serial -> pool offset
    const int n3 = class_weights(cp.key);
    for (int idx : cp.members) {
        const Triple& t = tr[idx];
        VolDesc a = make_desc(t.j, std::min(cp.tz, t.j.Z), g);
        auto it = woff.find(t.f->serial);
        if (it == woff.end()) {
            const uint32_t off = (uint32_t)wf.size();
            wf.resize(wf.size() + n3);
            wi.resize(wi.size() + n3);
            it = woff.emplace(t.f->serial, off).first;
        }
        a.woff = it->second;
        descs.push_back(a);
    }
    items = make_items(descs, cp.members, cp.key.k);
}

// Device copies of the weights go into the pools with device-to-device
// copies (the filters' weights live on the device).
hipError_t upload_class(const std::vector<Triple>& tr, ClassPlan& cp, char* base,
                        const std::vector<VolDesc>& descs, const std::vector<WorkItem>& items)
{
    hipError_t e = hipMemcpy(base + cp.off_desc, descs.data(), descs.size() * sizeof(VolDesc),
                             hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(base + cp.off_items, items.data(), items.size() * sizeof(WorkItem),
                      hipMemcpyHostToDevice);
    const int n3 = class_weights(cp.key);
    for (size_t m = 0; m < cp.members.size() && e == hipSuccess; ++m) {
        const vktFilter_* f = tr[cp.members[m]].f;
        const uint32_t off = descs[m].woff;
        if (cp.key.path == 2) {
            e = hipMemcpy(base + cp.off_wi + off * sizeof(int32_t), f->d_wq,
                          n3 * sizeof(uint32_t), hipMemcpyDeviceToDevice);
            continue;
        }
        e = hipMemcpy(base + cp.off_wf + off * sizeof(float), f->d_wf, n3 * sizeof(float),
                      hipMemcpyDeviceToDevice);
        if (e == hipSuccess && f->d_wi)
            e = hipMemcpy(base + cp.off_wi + off * sizeof(int32_t), f->d_wi,
                          n3 * sizeof(int32_t), hipMemcpyDeviceToDevice);
    }
    cp.nitems = (uint32_t)items.size();
    cp.args.vols = reinterpret_cast<const VolDesc*>(base + cp.off_desc);
    cp.args.items = reinterpret_cast<const WorkItem*>(base + cp.off_items);
    cp.args.nitems = cp.nitems;
    cp.args.counters = reinterpret_cast<uint32_t*>(base + cp.off_cnt);
    cp.args.wpool = reinterpret_cast<const float*>(base + cp.off_wf);
    cp.args.wipool = reinterpret_cast<const int32_t*>(base + cp.off_wi);
    return e;
}

hipError_t launch_class(const ClassPlan& cp, hipStream_t s)
{
    BatchArgs a = cp.args;
    void* params[] = {&a};
    return hipLaunchKernel(cp.func, dim3(cp.grid), dim3(256), params, 0, s);
}

// Time one class alone at a given slab depth (two launches on the caller's
// stream, the second timed; waits for both).
float time_class(const std::vector<Triple>& tr, ClassPlan& cp, char* base, int tz, int variant,
                 hipStream_t s)
{
    cp.tz = tz;
    cp.variant = variant;
    cp.func = class_kernel(cp.key, variant);
    int per_cu = 0, cus = 0, dev = 0;
    (void)hipGetDevice(&dev);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, cp.func, 256, 0) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 1;
    cp.grid = (unsigned)(per_cu * cus);
    std::vector<VolDesc> descs;
    std::vector<WorkItem> items;
    std::vector<float> wf;
    std::vector<int32_t> wi;
    class_arrays(tr, cp, descs, items, wf, wi);
    if (upload_class(tr, cp, base, descs, items) != hipSuccess) return -1.f;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return -1.f;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return -1.f;
    }
    float ms = -1.f;
    if (launch_class(cp, s) == hipSuccess && hipEventRecord(e0, s) == hipSuccess &&
        launch_class(cp, s) == hipSuccess && hipEventRecord(e1, s) == hipSuccess &&
        hipEventSynchronize(e1) == hipSuccess)
        (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ms;
}

vktError build_plan(const std::vector<Triple>& tr, std::vector<uintptr_t>&& sig, bool tune,
                    hipStream_t stream, std::shared_ptr<Plan>& out)
{
    auto plan = std::make_shared<Plan>();
    plan->sig = std::move(sig);
    if (hipGetDevice(&plan->device) != hipSuccess) return vktDeviceError;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, plan->device) !=
        hipSuccess)
        return vktDeviceError;

    std::map<ClassKey, std::vector<int>> groups;
    for (size_t i = 0; i < tr.size(); ++i) groups[tr[i].key].push_back((int)i);

    // size the device buffer for the most items any candidate makes (the
    // shorter tile variant at its smallest slab depth), so tuning and the
    // final plan fit
    size_t bytes = 0;
    for (auto& g : groups) {
        ClassPlan cp;
        cp.key = g.first;
        cp.members = g.second;
        cp.func = class_kernel(cp.key, 0);
        if (!cp.func) return vktUnsupported;
        size_t nitems = 0;
        for (int v = 0; v < kTileVariants; ++v) {
            const ClassGeom geom = class_geom(cp.key, v);
            size_t n = 0;
            for (int idx : cp.members) {
                const FilterJob& j = tr[idx].j;
                const int tzmin = std::min(geom.tz_min, j.Z);
                n += (size_t)((j.X + geom.tx - 1) / geom.tx) * ((j.Y + geom.ty - 1) / geom.ty) *
                     ((j.Z + tzmin - 1) / tzmin);
            }
            nitems = std::max(nitems, n);
        }
        const size_t n3 = (size_t)class_weights(cp.key);
        cp.off_desc = bytes = align_up(bytes, 256);
        bytes += cp.members.size() * sizeof(VolDesc);
        cp.off_items = bytes = align_up(bytes, 256);
        bytes += nitems * sizeof(WorkItem);
        cp.off_cnt = bytes = align_up(bytes, 256);
        bytes += 2 * sizeof(uint32_t);
        cp.off_wf = bytes = align_up(bytes, 256);
        bytes += (cp.members.size() * n3 + kWeightPad) * sizeof(float);
        cp.off_wi = bytes = align_up(bytes, 256);
        bytes += (cp.members.size() * n3 + kWeightPad) * sizeof(int32_t);
        plan->classes.push_back(cp);
    }
    plan->dbytes = bytes;
    hipError_t e = hipMalloc(&plan->dbuf, bytes);
    if (e != hipSuccess) return from_hip(e);
    e = hipMemset(plan->dbuf, 0, bytes);  // queue counters start at zero
    if (e != hipSuccess) return from_hip(e);

    for (auto& cp : plan->classes) {
        const TuneKey tk = tune_key(tr, cp);
        TuneVal tv = tuned(tk);
        if (tv.tz == 0 && tune) {
            // autotune: time every tile variant at candidate slab depths on
            // the real batch
            float best = -1.f;
            for (int v = 0; v < kTileVariants; ++v) {
                const ClassGeom geom = class_geom(cp.key, v);
                for (int cand : {8, 16, 32, 64}) {
                    if (cand < geom.tz_min && cand != 64) continue;
                    const float ms = time_class(tr, cp, plan->dbuf, std::max(cand, geom.tz_min),
                                                v, stream);
                    if (ms > 0.f && (best < 0.f || ms < best)) {
                        best = ms;
                        tv = TuneVal{std::max(cand, geom.tz_min), v};
                    }
                }
            }
            if (tv.tz > 0) {
                std::lock_guard<std::mutex> lk(g_tune_mu);
                g_tune[tk] = tv;
                tune_store_locked();
            }
        }
        cp.variant = tv.tz > 0 ? tv.variant : 0;
        const ClassGeom geom = class_geom(cp.key, cp.variant);
        cp.tz = std::max(tv.tz > 0 ? tv.tz : default_tz(cp.key, geom), geom.tz_min);
        cp.func = class_kernel(cp.key, cp.variant);
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, cp.func, 256, 0) !=
                hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        cp.grid = (unsigned)(per_cu * cus);
        std::vector<VolDesc> descs;
        std::vector<WorkItem> items;
        std::vector<float> wf;
        std::vector<int32_t> wi;
        class_arrays(tr, cp, descs, items, wf, wi);
        e = upload_class(tr, cp, plan->dbuf, descs, items);
        if (e != hipSuccess) return from_hip(e);
        if (cp.grid > cp.nitems) cp.grid = cp.nitems > 0 ? cp.nitems : 1;
    }

    // one graph: the class kernels as independent (parallel) kernel nodes
    e = hipGraphCreate(&plan->graph, 0);
    for (auto& cp : plan->classes) {
        if (e != hipSuccess) break;
        hipKernelNodeParams p{};
        void* params[] = {&cp.args};
        p.func = const_cast<void*>(cp.func);
        p.gridDim = dim3(cp.grid);
        p.blockDim = dim3(256);
        p.sharedMemBytes = 0;
        p.kernelParams = params;
        p.extra = nullptr;
        hipGraphNode_t node;
        e = hipGraphAddKernelNode(&node, plan->graph, nullptr, 0, &p);
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&plan->done, hipEventDisableTiming);
    if (e != hipSuccess) return from_hip(e);

    out = plan;
    std::shared_ptr<Plan> evicted;  // released after the lock (hipFree waits)
    {
        std::lock_guard<std::mutex> lk(g_plan_mu);
        if (g_plans.size() >= kMaxPlans) {
            evicted = std::move(g_plans.front());
            g_plans.erase(g_plans.begin());
        }
        g_plans.push_back(std::move(plan));
    }
    return vktNoError;
}

// Validate and plan every triple of a batch exactly as vktApplyFilter would,
// check that no output overlaps any volume of the batch, and collect the
// batch signature (the plan cache key).
vktError prepare_batch(int32_t n, const vktStructuredVolume* dst, const vktStructuredVolume* src,
                       const vktFilter* filters, vktAddressMode mode, vktPrecision prec,
                       hipStream_t stream, std::vector<Triple>& tr, std::vector<uintptr_t>& sig)
{
    tr.assign(n, Triple{});
    sig.clear();
    sig.reserve(4 + 6 * (size_t)n);
    sig.push_back((uintptr_t)n);
    sig.push_back((uintptr_t)mode);
    sig.push_back((uintptr_t)prec);
    sig.push_back((uintptr_t)thread_row_pair_min_cells());
    sig.push_back((uintptr_t)stream);
    for (int i = 0; i < n; ++i) {
        bool mfma = false, six = false;
        // (the batched form always runs the dense arithmetic)
        const vktError e =
            build_job(dst[i], src[i], filters[i], mode, prec, tr[i].j, mfma, six, nullptr, false);
        if (e != vktNoError) return e;
        const FilterJob& j = tr[i].j;
        tr[i].f = filters[i];
        if (mfma)
            tr[i].key = ClassKey{(int)j.fmt, j.k, 1, (six ? 1 : 0) | (mfma_row_pairs(j, six) ? 2 : 0)};
        else if (j.dot4) tr[i].key = ClassKey{(int)j.fmt, j.k, 2, j.q_signed ? 1 : 0};
        else tr[i].key = ClassKey{(int)j.fmt, j.k, 0, j.int_acc ? 1 : 0};
        sig.push_back((uintptr_t)j.src);
        sig.push_back((uintptr_t)j.dst);
        sig.push_back((uintptr_t)filters[i]->serial);
        sig.push_back((uintptr_t)j.X);
        sig.push_back((uintptr_t)j.Y);
        sig.push_back((uintptr_t)j.Z | ((uintptr_t)j.fmt << 40));
    }
    // outputs must not overlap any volume of the batch (they run concurrently)
    std::vector<std::pair<uintptr_t, uintptr_t>> dr, sr;
    for (int i = 0; i < n; ++i) {
        const uintptr_t b = (uintptr_t)cell_bytes(tr[i].j.fmt) * tr[i].j.X * tr[i].j.Y * tr[i].j.Z;
        dr.push_back({(uintptr_t)tr[i].j.dst, (uintptr_t)tr[i].j.dst + b});
        sr.push_back({(uintptr_t)tr[i].j.src, (uintptr_t)tr[i].j.src + b});
    }
    std::sort(dr.begin(), dr.end());
    for (size_t i = 1; i < dr.size(); ++i)
        if (dr[i].first < dr[i - 1].second) return vktInvalidValue;
    // sources sorted by start with the running maximum of their ends: an
    // output [a, b) meets a source iff some source starting before b ends
    // after a
    std::sort(sr.begin(), sr.end());
    std::vector<uintptr_t> max_end(sr.size());
    for (size_t i = 0; i < sr.size(); ++i)
        max_end[i] = std::max(sr[i].second, i ? max_end[i - 1] : (uintptr_t)0);
    for (const auto& d : dr) {
        const size_t m = (size_t)(std::lower_bound(sr.begin(), sr.end(),
                                                   std::make_pair(d.second, (uintptr_t)0)) -
                                  sr.begin());
        if (m > 0 && max_end[m - 1] > d.first) return vktInvalidValue;
    }
    return vktNoError;
}

// ---- allocation-free form ---------------------------------------------------
//
// The batch's descriptors, work lists, work-queue counters and weight pools
// go to this file-scope device array instead of a plan buffer.  Host code
// never passes the array's name to a kernel or a copy (on the host it is a
// stand-in, not a device address): it uses the address that
// hipGetSymbolAddress returns for the current device, looked up once per
// device.
constexpr size_t kNoAllocBytes = size_t(8) << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

struct NoAllocDevice {
    unsigned char* ptr = nullptr;       // this device's copy of `scratch`
    std::vector<unsigned char> staging; // host image of the array's head
    hipEvent_t copied = nullptr;        // the last upload from `staging` is done
    bool pending = false;
    std::mutex mu;                      // one call per device at a time (host side)
};
std::mutex g_noalloc_mu;
std::map<int, std::unique_ptr<NoAllocDevice>> g_noalloc;

// Set-up on the first call on a device, with that device current.
vktError noalloc_device(int dev, NoAllocDevice*& out)
{
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    auto it = g_noalloc.find(dev);
    if (it == g_noalloc.end()) {
        auto d = std::make_unique<NoAllocDevice>();
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return vktDeviceError;
        e = hipEventCreateWithFlags(&d->copied, hipEventDisableTiming);
        if (e != hipSuccess) return vktDeviceError;
        d->ptr = static_cast<unsigned char*>(p);
        d->staging.resize(kNoAllocBytes);
        it = g_noalloc.emplace(dev, std::move(d)).first;
    }
    out = it->second.get();
    return vktNoError;
}

vktError batched_no_alloc(const std::vector<Triple>& tr, hipStream_t stream)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return vktDeviceError;
    NoAllocDevice* nd = nullptr;
    vktError ve = noalloc_device(dev, nd);
    if (ve != vktNoError) return ve;

    // plan every class as the cached form does (same tile variants and slab
    // depths: the tuning table's entry, else the defaults; this form never
    // times candidates)
    std::map<ClassKey, std::vector<int>> groups;
    for (size_t i = 0; i < tr.size(); ++i) groups[tr[i].key].push_back((int)i);
    std::vector<ClassPlan> classes;
    std::vector<std::vector<VolDesc>> descs(groups.size());
    std::vector<std::vector<WorkItem>> items(groups.size());
    std::vector<size_t> npool(groups.size());
    // layout: the heads of all classes (descriptors, work list, counters),
    // then the weight pools
    size_t bytes = 0, c = 0;
    for (auto& g : groups) {
        ClassPlan cp;
        cp.key = g.first;
        cp.members = g.second;
        const TuneVal tv = tuned(tune_key(tr, cp));
        cp.variant = tv.tz > 0 ? tv.variant : 0;
        cp.func = class_kernel(cp.key, cp.variant);
        if (!cp.func) return vktUnsupported;
        const ClassGeom geom = class_geom(cp.key, cp.variant);
        cp.tz = std::max(tv.tz > 0 ? tv.tz : default_tz(cp.key, geom), geom.tz_min);
        std::vector<float> wf;
        std::vector<int32_t> wi;
        class_arrays(tr, cp, descs[c], items[c], wf, wi);
        const size_t n3 = (size_t)class_weights(cp.key);
        for (const auto& d : descs[c]) npool[c] = std::max(npool[c], (size_t)d.woff / n3 + 1);
        cp.off_desc = bytes = align_up(bytes, 256);
        bytes += descs[c].size() * sizeof(VolDesc);
        cp.off_items = bytes = align_up(bytes, 256);
        bytes += items[c].size() * sizeof(WorkItem);
        cp.off_cnt = bytes = align_up(bytes, 256);
        bytes += 2 * sizeof(uint32_t);
        cp.grid = (unsigned)resident_wgs(cp.func);
        classes.push_back(cp);
        ++c;
    }
    for (size_t i = 0; i < classes.size(); ++i) {
        ClassPlan& cp = classes[i];
        const size_t n3 = (size_t)class_weights(cp.key);
        cp.off_wf = bytes = align_up(bytes, 256);
        bytes += (npool[i] * n3 + kWeightPad) * sizeof(float);
        cp.off_wi = bytes = align_up(bytes, 256);
        bytes += (npool[i] * n3 + kWeightPad) * sizeof(int32_t);
    }
    if (bytes > kNoAllocBytes) return vktUnsupported;  // the batch does not fit

    std::lock_guard<std::mutex> lk(nd->mu);
    // the previous upload must have read the staging image before it changes
    if (nd->pending && hipEventSynchronize(nd->copied) != hipSuccess) return vktDeviceError;
    nd->pending = false;
    // image of the used region: descriptors, work lists, zeroed counters and
    // zeroed weight pools (the upload clears the counters and the pools' pads;
    // the weights come from the filters' device buffers below)
    std::memset(nd->staging.data(), 0, bytes);
    for (size_t i = 0; i < classes.size(); ++i) {
        const ClassPlan& cp = classes[i];
        std::memcpy(&nd->staging[cp.off_desc], descs[i].data(), descs[i].size() * sizeof(VolDesc));
        std::memcpy(&nd->staging[cp.off_items], items[i].data(),
                    items[i].size() * sizeof(WorkItem));
    }
    hipError_t e =
        hipMemcpyAsync(nd->ptr, nd->staging.data(), bytes, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipEventRecord(nd->copied, stream);
    if (e != hipSuccess) return from_hip(e);
    nd->pending = true;
    for (size_t i = 0; i < classes.size() && e == hipSuccess; ++i) {
        ClassPlan& cp = classes[i];
        const size_t n3 = (size_t)class_weights(cp.key);
        std::map<uint32_t, const vktFilter_*> pool;
        for (size_t m = 0; m < cp.members.size(); ++m)
            pool.emplace(descs[i][m].woff, tr[cp.members[m]].f);
        for (const auto& pf : pool) {
            const vktFilter_* f = pf.second;
            const uint32_t off = pf.first;
            if (cp.key.path == 2) {
                e = hipMemcpyAsync(nd->ptr + cp.off_wi + off * sizeof(int32_t), f->d_wq,
                                   n3 * sizeof(uint32_t), hipMemcpyDeviceToDevice, stream);
            } else {
                e = hipMemcpyAsync(nd->ptr + cp.off_wf + off * sizeof(float), f->d_wf,
                                   n3 * sizeof(float), hipMemcpyDeviceToDevice, stream);
                if (e == hipSuccess && f->d_wi)
                    e = hipMemcpyAsync(nd->ptr + cp.off_wi + off * sizeof(int32_t), f->d_wi,
                                       n3 * sizeof(int32_t), hipMemcpyDeviceToDevice, stream);
            }
            if (e != hipSuccess) break;
        }
        cp.nitems = (uint32_t)items[i].size();
        cp.args.vols = reinterpret_cast<const VolDesc*>(nd->ptr + cp.off_desc);
        cp.args.items = reinterpret_cast<const WorkItem*>(nd->ptr + cp.off_items);
        cp.args.nitems = cp.nitems;
        cp.args.counters = reinterpret_cast<uint32_t*>(nd->ptr + cp.off_cnt);
        cp.args.wpool = reinterpret_cast<const float*>(nd->ptr + cp.off_wf);
        cp.args.wipool = reinterpret_cast<const int32_t*>(nd->ptr + cp.off_wi);
        if (cp.grid > cp.nitems) cp.grid = cp.nitems > 0 ? cp.nitems : 1;
        if (e == hipSuccess) e = launch_class(cp, stream);
    }
    return from_hip(e);
}

}  // namespace
}  // namespace vkt

extern "C" {

vktError vktApplyFilterBatched(int32_t n, const vktStructuredVolume* dst,
                               const vktStructuredVolume* src, const vktFilter* filters,
                               vktAddressMode mode)
{
    using namespace vkt;
    if (n < 0 || (n > 0 && (!dst || !src || !filters))) return vktInvalidValue;
    if (n == 0) return vktNoError;
    const vktPrecision prec = thread_precision();
    hipStream_t stream = thread_stream();
    std::vector<Triple> tr;
    std::vector<uintptr_t> sig;
    const vktError ve = prepare_batch(n, dst, src, filters, mode, prec, stream, tr, sig);
    if (ve != vktNoError) return ve;

    std::lock_guard<std::mutex> serial(g_batch_mu);
    std::shared_ptr<Plan> plan;
    {
        int dev = 0;
        (void)hipGetDevice(&dev);
        std::lock_guard<std::mutex> lk(g_plan_mu);
        for (auto it = g_plans.begin(); it != g_plans.end(); ++it)
            if ((*it)->sig == sig && (*it)->device == dev) {
                plan = *it;
                g_plans.erase(it);        // a hit becomes the most recently used
                g_plans.push_back(plan);
                break;
            }
    }
    if (!plan) {
        const vktError e = build_plan(tr, std::move(sig), thread_autotune(), stream, plan);
        if (e != vktNoError) return e;
    }
    hipError_t e = hipGraphLaunch(plan->exec, stream);
    if (e == hipSuccess) e = hipEventRecord(plan->done, stream);
    return from_hip(e);
}

vktError vktApplyFilterBatchedNoAlloc(int32_t n, const vktStructuredVolume* dst,
                                      const vktStructuredVolume* src, const vktFilter* filters,
                                      vktAddressMode mode)
{
    using namespace vkt;
    if (n < 0 || (n > 0 && (!dst || !src || !filters))) return vktInvalidValue;
    if (n == 0) return vktNoError;
    hipStream_t stream = thread_stream();
    std::vector<Triple> tr;
    std::vector<uintptr_t> sig;
    const vktError ve =
        prepare_batch(n, dst, src, filters, mode, thread_precision(), stream, tr, sig);
    if (ve != vktNoError) return ve;
    return batched_no_alloc(tr, stream);
}

}  // extern "C"
