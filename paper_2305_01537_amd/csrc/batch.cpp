// batch.cpp -- host side of the batched filter: many uneven spherical patches
// in one persistent kernel launch, replayed from a captured HIP graph, with a
// schedule picked by an autotuner and remembered in a JSON cache.
//
// The operation per patch is exactly the plan's (arXiv:2305.01537,
// Sec. II.A): theta-pass then phi-pass (forward), or the reverse (adjoint).
// What the batch adds is scheduling: every patch's theta groups and ring-pair
// groups become items of one work list (see batch_kernels.h), so small patches do
// not leave the GPU idle and one graph launch covers all of them.
#include "../../include/sphfilt.h"
#include "batch_internal.h"
#include "host_tables.h"
#include "tune_cache.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <new>
#include <sstream>
#include <string>
#include <vector>

using namespace sphfilt;

namespace {

constexpr int kMaxGraphs = 8;
constexpr int kSpinLimit = 1 << 20;   // ~0.1 s of polling per shell

struct PatchHost {
    int n_r, n_theta, n_phi, n_fields;
    HostTables tables;
    int theta_off = 0, phi_off = 0;   // into the concatenated item arrays
    int phi_rest_off = 0;             // the phi items of theta-idle shells
    int fc_off = 0;                   // fused shells' ring cutoffs
    int shell_base = 0;               // first global shell id
    int cols = 0;                     // theta sub-tile width (meridian pairs)
    long long n_points = 0;
};

struct ModeWork {
    bool built = false;
    int n_work = 0, n_first = 0;
    int n_indep = 0;        // second-pass items at [n_first, n_first + n_indep) touch no
                            // shell a first-pass item writes
    BatchWork *d_work = nullptr;
    int *d_shells = nullptr;
    int *d_need = nullptr;
};

struct GraphEntry {
    int mode = 0, split = 0, wpc = 0;
    int wait_fault = 0;       // captured with the forced give-up of SPHFILT_FAULT=wait
    std::vector<const double *> ins;
    std::vector<double *> outs;
    const double **d_ins = nullptr;
    double **d_outs = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t last_use = 0;
};

// Where a call's counters, tickets, error word and pointer tables live: the
// batch's own device memory (graph path) or the static scratch array of the
// allocation-free entry point.
struct CallScratch {
    int *counters;
    int *tickets;
    int *error;
    const double *const *ins;
    double *const *outs;
};

}  // namespace

struct sphfilt_batch_s {
    int device = 0;
    int n_cu = 0;
    int max_wpc = 1;
    std::string arch;
    uint64_t signature = 0;
    std::vector<PatchHost> patches;
    ThetaItem *d_th = nullptr;
    PhiItem *d_ph = nullptr;
    double *d_fc = nullptr;
    int fused = 1;                     // fused items for patches that allow them
    BatchPatchDev *d_patches = nullptr;
    double *d_eneg = nullptr;
    std::map<int, Twiddle *> d_tw;
    int n_shells_total = 0;
    int *d_counters = nullptr;
    int *d_tickets = nullptr;
    int *d_error = nullptr;
    ModeWork modes[4];
    std::vector<GraphEntry> graphs;
    int split = 0, wpc = -1;           // schedule: see effective_wpc
    int theta_tiles = 1;               // meridian tiles per theta item
    int phi_groups = 1;                // workgroup rounds of ring pairs per phi item
    std::map<int, int> theta_cols;     // theta line length -> sub-tile width (tuned; else default)
    std::vector<BatchPatchDev> pdev;   // host copy of d_patches
    int hybrid = 0;                    // some patch has a hybrid field
    int variant = 0;                   // kernel instance: kBatchHybrid | kBatchMixedRadix
    double tuned_us = -1.0;
    double default_us = -1.0;          // the untuned schedule's time, measured by the tuner
    uint64_t clock = 0;
    hipStream_t capture_stream = nullptr;
    hipStream_t side_stream = nullptr;    // parallel branch of split = 2 graphs
    hipEvent_t fork = nullptr, join = nullptr;
    unsigned char *noalloc = nullptr;     // device address of the static scratch array
    int last_noalloc = 0;                 // the last call went through the allocation-free entry
};

namespace {

uint64_t signature(const std::string &arch, int n_patches, const sphfilt_patch_desc *d)
{
    auto fnv = fnv1a;
    uint64_t h = kFnvSeed;
    const char tag[] = "batch";
    h = fnv(h, tag, sizeof(tag));
    h = fnv(h, arch.data(), arch.size());
    h = fnv(h, &n_patches, sizeof(n_patches));
    for (int p = 0; p < n_patches; ++p) {
        const int dims[4] = {d[p].n_r, d[p].n_theta, d[p].n_phi, d[p].n_fields};
        h = fnv(h, dims, sizeof(dims));
        h = fnv(h, d[p].parity, sizeof(int) * d[p].n_fields);
        h = fnv(h, d[p].cut.L, sizeof(double) * d[p].n_fields);
        const int has[2] = {d[p].cut.rho != nullptr, d[p].cut.kind != nullptr};
        h = fnv(h, has, sizeof(has));
        if (d[p].cut.rho) h = fnv(h, d[p].cut.rho, sizeof(double) * d[p].n_r);
        if (d[p].cut.kind) h = fnv(h, d[p].cut.kind, sizeof(int) * d[p].n_fields);
        h = fnv(h, &d[p].cut.floor_modes, sizeof(double));
        h = fnv(h, &d[p].cut.detector_eps, sizeof(double));
        h = fnv(h, &d[p].cut.detector_threshold, sizeof(double));
    }
    return h;
}

// ---- work lists ----------------------------------------------------------
void add_pass(const sphfilt_batch b, int pi, bool theta, bool all, bool second,
              std::vector<BatchWork> *work, std::vector<int> *shells)
{
    const PatchHost &p = b->patches[(size_t)pi];
    if (theta) {
        // groups of S shells; each item takes up to theta_tiles meridian tiles
        const int n = all ? (int)p.tables.theta.size() : p.tables.theta_active;
        const int C = theta_lines_per_group(2 * p.n_theta);
        const int S = C / p.cols;
        const int T = (p.n_phi / 2) / (2 * p.cols);
        const int TI = std::max(1, std::min(b->theta_tiles, T));
        for (int g = 0; g * S < n; ++g) {
            const int nv = std::min(S, n - g * S);
            const int off = (int)shells->size();
            for (int u = 0; u < nv; ++u)
                shells->push_back(p.shell_base + p.tables.theta[(size_t)(g * S + u)].shell);
            for (int tile = 0; tile < T; tile += TI)
                work->push_back(BatchWork{pi, 0, (int16_t)second, p.theta_off + g * S, (int16_t)nv,
                                          (int16_t)tile, off, nv, 0, std::min(TI, T - tile)});
        }
    } else {
        // up to phi_groups workgroup rounds of L ring pairs per item
        const int n = all ? (int)p.tables.phi.size() : p.tables.phi_active;
        const int L = default_phi_lines(p.n_phi) * std::max(1, b->phi_groups);
        for (int c = 0; c * L < n; ++c) {
            const int nv = std::min(L, n - c * L);
            std::vector<int> s;
            for (int u = 0; u < nv; ++u)
                s.push_back(p.shell_base + p.tables.phi[(size_t)(c * L + u)].ring / p.n_theta);
            std::sort(s.begin(), s.end());
            s.erase(std::unique(s.begin(), s.end()), s.end());
            const int off = (int)shells->size();
            shells->insert(shells->end(), s.begin(), s.end());
            work->push_back(BatchWork{pi, 1, (int16_t)second, p.phi_off + c * L, (int16_t)nv, 0, off,
                                      (int)s.size(), 0, 1});
        }
    }
}

// Lines that are not powers of two (48, 80, 96, 160, 192) take the batch
// kernel's second instance.
bool mixed_radix_line(int n) { return (n & (n - 1)) != 0; }

// A patch whose theta-filtered shells are all fused (n_phi = 2 n_theta in {32, 64, 128},
// see build_items) runs entirely in the first pass: groups of whole shells
// (both passes, add_fused_shells), and the ring pairs of its theta-idle shells
// (add_rest_rings; out of place also their identity rings, copied).  Nothing
// waits for these items.
bool patch_fused(const sphfilt_batch b, const PatchHost &p)
{
    return b->fused && p.tables.n_fused > 0 && p.tables.n_fused == p.tables.theta_active;
}

void add_fused_shells(const sphfilt_batch b, int pi, bool adjoint, std::vector<BatchWork> *work)
{
    const PatchHost &p = b->patches[(size_t)pi];
    const int S = shells_per_group(p.n_phi), lines = p.n_theta / 2;
    for (int g = 0; g * S < p.tables.n_fused; ++g) {
        const int nv = std::min(S, p.tables.n_fused - g * S);
        work->push_back(BatchWork{pi, 2, 0, p.theta_off + g * S, (int16_t)nv, (int16_t)adjoint, 0, 0,
                                  p.fc_off + g * S * lines, 1});
    }
}

void add_rest_rings(const sphfilt_batch b, int pi, bool all, std::vector<BatchWork> *work)
{
    const PatchHost &p = b->patches[(size_t)pi];
    const int n = all ? (int)p.tables.phi_rest.size() : p.tables.phi_rest_active;
    const int L = default_phi_lines(p.n_phi) * std::max(1, b->phi_groups);
    for (int c = 0; c * L < n; ++c)
        work->push_back(BatchWork{pi, 1, 0, p.phi_rest_off + c * L, (int16_t)std::min(L, n - c * L), 0,
                                  0, 0, 0, 1});
}

int build_mode(sphfilt_batch b, int mode)
{
    ModeWork &m = b->modes[mode];
    if (m.built) return SPHFILT_OK;
    const bool adjoint = mode & 1, inplace = mode & 2;
    std::vector<BatchWork> work;
    std::vector<int> shells;
    // fused shell groups first: they hold a workgroup longest (a whole shell,
    // both passes), so they start before the short items rather than trail them
    for (int p = 0; p < (int)b->patches.size(); ++p)
        if (patch_fused(b, b->patches[(size_t)p])) add_fused_shells(b, p, adjoint, &work);
    for (int p = 0; p < (int)b->patches.size(); ++p) {
        if (patch_fused(b, b->patches[(size_t)p]))
            add_rest_rings(b, p, !inplace, &work);
        else
            add_pass(b, p, !adjoint, !inplace, false, &work, &shells);
    }
    const int n_first = (int)work.size();
    std::vector<BatchWork> second;
    for (int p = 0; p < (int)b->patches.size(); ++p)
        if (!patch_fused(b, b->patches[(size_t)p]))
            add_pass(b, p, adjoint, false, true, &second, &shells);
    std::vector<int> need((size_t)std::max(1, b->n_shells_total), 0);
    for (int k = 0; k < n_first; ++k)
        for (int i = 0; i < work[(size_t)k].n_shells; ++i) ++need[(size_t)shells[(size_t)(work[(size_t)k].shell_off + i)]];
    // second-pass items whose shells no first-pass item writes (in place: the
    // rings of theta-idle shells in the forward order) come first: they need
    // not wait, and split = 2 runs them on a parallel branch
    auto independent = [&](const BatchWork &w) {
        for (int i = 0; i < w.n_shells; ++i)
            if (need[(size_t)shells[(size_t)(w.shell_off + i)]] > 0) return false;
        return true;
    };
    std::stable_partition(second.begin(), second.end(), independent);
    int n_indep = 0;
    while (n_indep < (int)second.size() && independent(second[(size_t)n_indep])) ++n_indep;
    work.insert(work.end(), second.begin(), second.end());
    int rc = upload(&m.d_work, work);
    if (!rc) rc = upload(&m.d_shells, shells);
    if (!rc) rc = upload(&m.d_need, need);
    if (rc) return rc;
    m.n_work = (int)work.size();
    m.n_first = n_first;
    m.n_indep = n_indep;
    m.built = true;
    return SPHFILT_OK;
}

void free_graph(GraphEntry *g)
{
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->d_ins) (void)hipFree((void *)g->d_ins);
    if (g->d_outs) (void)hipFree((void *)g->d_outs);
    *g = GraphEntry{};
}

// wpc < 0: one workgroup per item; 0: persistent, as many as fit; k: k per CU.
int effective_wpc(sphfilt_batch b, int wpc)
{
    if (wpc < 0) return -1;
    return wpc == 0 || wpc > b->max_wpc ? b->max_wpc : wpc;
}

// SPHFILT_FAULT=wait (tests only): every wait target is raised by one and the
// spin is cut short, so that second-pass items of the one-kernel schedule give
// up at once; the kernels still run to their end.
constexpr int kFaultSpinLimit = 64;

// Enqueue the reset kernel and the persistent kernel(s) of `m` on stream s
// (a capture stream, or the caller's stream for the allocation-free call).
int record(sphfilt_batch b, const ModeWork &m, int split, int wpc_setting, const CallScratch &sc,
           int wait_fault, hipStream_t s)
{
    const int wpc = effective_wpc(b, wpc_setting);
    const int grid = wpc < 0 ? 0 : wpc * b->n_cu;
    const int spin = wait_fault ? kFaultSpinLimit : kSpinLimit, bias = wait_fault ? 1 : 0;
    auto go = [&](int first, int n, int *ticket, int deps, hipStream_t st) {
        return launch_batch(grid, m.d_work + first, n, b->d_patches, sc.ins, sc.outs, b->d_th,
                            b->d_ph, b->d_fc, m.d_shells, sc.counters, m.d_need, ticket, sc.error,
                            b->d_eneg, deps, spin, bias, b->variant, st);
    };
    hipError_t e = launch_batch_reset(sc.counters, b->n_shells_total, sc.tickets, 3, sc.error, s);
    if (e != hipSuccess) return SPHFILT_EDEVICE;
    if (split == 2 && m.n_indep > 0) {
        // fork: the independent second-pass items on the side stream, the
        // first pass and then the dependent second-pass items here; join
        const int dep0 = m.n_first + m.n_indep;
        e = hipEventRecord(b->fork, s);
        if (e == hipSuccess) e = hipStreamWaitEvent(b->side_stream, b->fork, 0);
        if (e == hipSuccess) e = go(m.n_first, m.n_indep, sc.tickets + 2, 0, b->side_stream);
        if (e == hipSuccess) e = go(0, m.n_first, sc.tickets, 0, s);
        if (e == hipSuccess) e = go(dep0, m.n_work - dep0, sc.tickets + 1, 0, s);
        if (e == hipSuccess) e = hipEventRecord(b->join, b->side_stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, b->join, 0);
    } else if (split) {
        e = go(0, m.n_first, sc.tickets, 0, s);
        if (e == hipSuccess) e = go(m.n_first, m.n_work - m.n_first, sc.tickets + 1, 0, s);
    } else {
        e = go(0, m.n_work, sc.tickets, 1, s);
    }
    return e == hipSuccess ? SPHFILT_OK : SPHFILT_EDEVICE;
}

// The graph for (mode, pointers, schedule), captured on first use and cached.
int get_graph(sphfilt_batch b, int mode, const double *const *ins, double *const *outs,
              GraphEntry **out)
{
    const size_t P = b->patches.size();
    const int wait_fault = fault("wait") ? 1 : 0;
    for (GraphEntry &g : b->graphs) {
        if (g.mode != mode || g.split != b->split || g.wpc != b->wpc || g.wait_fault != wait_fault)
            continue;
        if (!std::equal(g.ins.begin(), g.ins.end(), ins) || !std::equal(g.outs.begin(), g.outs.end(), outs))
            continue;
        g.last_use = ++b->clock;
        *out = &g;
        return SPHFILT_OK;
    }
    int rc = build_mode(b, mode);
    if (rc) return rc;
    if ((int)b->graphs.size() >= kMaxGraphs) {
        auto lru = std::min_element(b->graphs.begin(), b->graphs.end(),
                                    [](const GraphEntry &x, const GraphEntry &y) { return x.last_use < y.last_use; });
        free_graph(&*lru);
        b->graphs.erase(lru);
    }
    GraphEntry g;
    g.mode = mode;
    g.split = b->split;
    g.wpc = b->wpc;
    g.wait_fault = wait_fault;
    g.ins.assign(ins, ins + P);
    g.outs.assign(outs, outs + P);
    rc = upload(&g.d_ins, g.ins);
    if (!rc) rc = upload(&g.d_outs, g.outs);
    if (!rc) {
        hipError_t e = hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) rc = SPHFILT_EDEVICE;
        if (!rc) {
            const CallScratch sc{b->d_counters, b->d_tickets, b->d_error, g.d_ins, g.d_outs};
            const int rr = record(b, b->modes[mode], g.split, g.wpc, sc, g.wait_fault,
                                  b->capture_stream);
            e = hipStreamEndCapture(b->capture_stream, &g.graph);
            rc = rr ? rr : (e == hipSuccess ? SPHFILT_OK : SPHFILT_EDEVICE);
        }
        if (!rc && hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0) != hipSuccess)
            rc = SPHFILT_EDEVICE;
    }
    if (rc) {
        free_graph(&g);
        return rc;
    }
    g.last_use = ++b->clock;
    b->graphs.push_back(g);
    *out = &b->graphs.back();
    return SPHFILT_OK;
}

// Drop the captured graphs and the work lists (rebuilt on the next call).
void free_work(sphfilt_batch b)
{
    for (GraphEntry &g : b->graphs) free_graph(&g);
    b->graphs.clear();
    for (ModeWork &m : b->modes) {
        if (m.d_work) (void)hipFree(m.d_work);
        if (m.d_shells) (void)hipFree(m.d_shells);
        if (m.d_need) (void)hipFree(m.d_need);
        m = ModeWork{};
    }
}

// Build the work lists of all four modes (forward/adjoint x in/out of place)
// up front, so that no call has to allocate them.
int ensure_modes(sphfilt_batch b)
{
    for (int mode = 0; mode < 4; ++mode) {
        const int rc = build_mode(b, mode);
        if (rc) return rc;
    }
    return SPHFILT_OK;
}

void free_batch(sphfilt_batch b)
{
    free_work(b);
    for (auto &kv : b->d_tw) (void)hipFree(kv.second);
    b->d_tw.clear();
    void *ptrs[] = {b->d_th, b->d_ph, b->d_fc, b->d_patches, b->d_eneg, b->d_counters, b->d_tickets,
                    b->d_error};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
    if (b->side_stream) (void)hipStreamDestroy(b->side_stream);
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->join) (void)hipEventDestroy(b->join);
}

int check_pointers(sphfilt_batch b, const double *const *ins, double *const *outs, bool *inplace)
{
    if (!ins || !outs) return SPHFILT_EINVAL;
    const size_t P = b->patches.size();
    bool all_in = true;
    for (size_t p = 0; p < P; ++p) {
        if (!ins[p] || !outs[p]) return SPHFILT_EINVAL;
        const uintptr_t a = (uintptr_t)ins[p], o = (uintptr_t)outs[p];
        const size_t n = sizeof(double) * (size_t)b->patches[p].n_points;
        if ((a | o) & 15) return SPHFILT_EINVAL;                           // 16-byte accesses
        if (a != o && a < o + n && o < a + n) return SPHFILT_EINVAL;
        if (a != o) all_in = false;
    }
    // no patch may write into another patch's input or output
    for (size_t p = 0; p < P; ++p) {
        const uintptr_t o = (uintptr_t)outs[p];
        const size_t n = sizeof(double) * (size_t)b->patches[p].n_points;
        for (size_t q = 0; q < P; ++q) {
            if (q == p) continue;
            const size_t nq = sizeof(double) * (size_t)b->patches[q].n_points;
            const uintptr_t oq = (uintptr_t)outs[q], iq = (uintptr_t)ins[q];
            if (o < oq + nq && oq < o + n) return SPHFILT_EINVAL;
            if (o < iq + nq && iq < o + n) return SPHFILT_EINVAL;
        }
    }
    *inplace = all_in;
    return SPHFILT_OK;
}

int launch(sphfilt_batch b, const double *const *ins, double *const *outs, int adjoint,
           hipStream_t stream)
{
    bool inplace = false;
    int rc = check_pointers(b, ins, outs, &inplace);
    if (rc) return rc;
    if (fault("launch")) return SPHFILT_EDEVICE;
    const int mode = (adjoint ? 1 : 0) | (inplace ? 2 : 0);
    GraphEntry *g = nullptr;
    rc = get_graph(b, mode, ins, outs, &g);
    if (rc) return rc;
    b->last_noalloc = 0;
    return hipGraphLaunch(g->exec, stream) == hipSuccess ? SPHFILT_OK : SPHFILT_EDEVICE;
}

// The allocation-free call: the batch's work lists (built at creation) and the
// static scratch array; the kernels are launched directly on the caller's
// stream (no graph, no allocation, no library routine that allocates).
int launch_noalloc(sphfilt_batch b, const double *const *ins, double *const *outs, int adjoint,
                   hipStream_t stream)
{
    bool inplace = false;
    int rc = check_pointers(b, ins, outs, &inplace);
    if (rc) return rc;
    if ((int)b->patches.size() > kNoAllocMaxPatches || b->n_shells_total > kNoAllocMaxShells)
        return SPHFILT_EUNSUPPORTED;
    if (!b->noalloc && noalloc_scratch(b->device, &b->noalloc) != hipSuccess) return SPHFILT_EDEVICE;
    if (fault("launch")) return SPHFILT_EDEVICE;
    const int mode = (adjoint ? 1 : 0) | (inplace ? 2 : 0);
    const ModeWork &m = b->modes[mode];
    if (!m.built) return SPHFILT_EINVAL;      // rebuilt by every call that drops them
    unsigned char *base = b->noalloc;
    int *head = reinterpret_cast<int *>(base);
    const CallScratch sc{reinterpret_cast<int *>(base + kNoAllocCounterOffset), head, head + 3,
                         reinterpret_cast<const double *const *>(base + kNoAllocPtrOffset),
                         reinterpret_cast<double *const *>(base + kNoAllocPtrOffset) + kNoAllocMaxPatches};
    if (noalloc_set_pointers(base, ins, outs, (int)b->patches.size(), stream) != hipSuccess)
        return SPHFILT_EDEVICE;
    b->last_noalloc = 1;
    return record(b, m, b->split, b->wpc, sc, fault("wait") ? 1 : 0, stream);
}

// Time the current schedule on scratch fields: the median over `reps` rounds
// of the time per call, each round kBatchCallsPerRound graph launches back to
// back, as a time-stepping loop makes them (one call at a time would expose
// each launch's latency).
constexpr int kBatchCallsPerRound = 3;

int time_schedule(sphfilt_batch b, const std::vector<double *> &bufs, hipStream_t s, int reps, double *us)
{
    std::vector<const double *> ins(bufs.begin(), bufs.end());
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return SPHFILT_EDEVICE;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return SPHFILT_EDEVICE; }
    std::vector<float> t;
    int rc = SPHFILT_OK;
    for (int r = 0; r < reps + 2 && !rc; ++r) {
        if (hipEventRecord(e0, s) != hipSuccess) { rc = SPHFILT_EDEVICE; break; }
        for (int c = 0; c < kBatchCallsPerRound && !rc; ++c) rc = launch(b, ins.data(), bufs.data(), 0, s);
        if (rc) break;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
            rc = SPHFILT_EDEVICE;
            break;
        }
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (r >= 2) t.push_back(ms / kBatchCallsPerRound);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    std::sort(t.begin(), t.end());
    *us = 1000.0 * t[t.size() / 2];
    return SPHFILT_OK;
}

// ---- schedules and the autotuner ----------------------------------------
// The supported theta line lengths, the index order of
// sphfilt_batch_schedule::theta_cols.
constexpr int kLines[9] = {32, 48, 64, 80, 96, 128, 160, 192, 256};

struct Sched {
    int fused = 1, split = 0, wpc = -1, theta_tiles = 1, phi_groups = 1;
    std::map<int, int> cols;      // theta line length -> sub-tile width (absent: default)
};

Sched current(const sphfilt_batch b)
{
    Sched c;
    c.fused = b->fused;
    c.split = b->split;
    c.wpc = b->wpc;
    c.theta_tiles = b->theta_tiles;
    c.phi_groups = b->phi_groups;
    c.cols = b->theta_cols;
    return c;
}

// The theta sub-tile width of patch p under the batch's tile table: the
// tuned width for its line length where the patch's grid takes it, else the
// default.
int patch_cols(const sphfilt_batch b, const PatchHost &p)
{
    auto it = b->theta_cols.find(2 * p.n_theta);
    if (it != b->theta_cols.end() && theta_shape_ok(2 * p.n_theta, it->second, p.n_phi)) return it->second;
    return default_theta_cols(2 * p.n_theta, p.n_phi);
}

// Make `c` the batch's schedule.  Work lists and graphs are dropped (and
// rebuilt) when the item shapes change; the patch table is re-uploaded when a
// tile width changes.  Synchronises the device in those cases.
int set_sched(sphfilt_batch b, const Sched &c)
{
    const bool shapes = c.fused != b->fused || c.theta_tiles != b->theta_tiles ||
                        c.phi_groups != b->phi_groups || c.cols != b->theta_cols;
    b->split = c.split;
    b->wpc = c.wpc;
    if (!shapes) return SPHFILT_OK;
    if (hipDeviceSynchronize() != hipSuccess) return SPHFILT_EDEVICE;
    free_work(b);
    b->fused = c.fused;
    b->theta_tiles = c.theta_tiles;
    b->phi_groups = c.phi_groups;
    b->theta_cols = c.cols;
    bool changed = false;
    for (size_t i = 0; i < b->patches.size(); ++i) {
        PatchHost &p = b->patches[i];
        const int cols = patch_cols(b, p);
        if (cols != p.cols) {
            p.cols = cols;
            b->pdev[i].cp_log2 = ilog2_int(cols);
            changed = true;
        }
    }
    if (changed && hipMemcpy(b->d_patches, b->pdev.data(), sizeof(BatchPatchDev) * b->pdev.size(),
                             hipMemcpyHostToDevice) != hipSuccess)
        return SPHFILT_EDEVICE;
    return ensure_modes(b);
}

TuneFields sched_fields(const sphfilt_batch b, const Sched &c, double us, double default_us)
{
    TuneFields f;
    f["what"] = tune_str("batch");
    f["arch"] = tune_str(b->arch);
    f["split"] = tune_num(c.split);
    f["wpc"] = tune_num(c.wpc);
    f["fused"] = tune_num(c.fused);
    f["theta_tiles"] = tune_num(c.theta_tiles);
    f["phi_groups"] = tune_num(c.phi_groups);
    std::string cols;
    for (const auto &kv : c.cols) cols += (cols.empty() ? "" : ",") + std::to_string(kv.first) + ":" + std::to_string(kv.second);
    f["theta_cols"] = tune_str(cols);
    f["us"] = tune_num(us);
    f["default_us"] = tune_num(default_us);
    return f;
}

bool sched_from_fields(const sphfilt_batch b, const TuneFields &f, Sched *c, double *us, double *def)
{
    Sched r;
    std::string what, cols;
    if (!tune_string(f, "what", &what) || what != "batch" || !tune_int(f, "split", &r.split) ||
        !tune_int(f, "wpc", &r.wpc) || !tune_int(f, "fused", &r.fused) ||
        !tune_int(f, "theta_tiles", &r.theta_tiles) || !tune_int(f, "phi_groups", &r.phi_groups) ||
        !tune_string(f, "theta_cols", &cols))
        return false;
    if (r.split < 0 || r.split > 2 || r.wpc < -1 || r.wpc > b->max_wpc || (r.fused != 0 && r.fused != 1) ||
        r.theta_tiles < 1 || r.theta_tiles > 8 || r.phi_groups < 1 || r.phi_groups > 8)
        return false;
    std::istringstream in(cols);
    std::string item;
    while (std::getline(in, item, ',')) {
        const size_t colon = item.find(':');
        if (colon == std::string::npos) return false;
        const int n = std::atoi(item.substr(0, colon).c_str()), w = std::atoi(item.c_str() + colon + 1);
        if (!supported_line(n) || (w != 4 && w != 8 && w != 16 && w != 32 && w != 64)) return false;
        r.cols[n] = w;
    }
    *c = r;
    if (!tune_double(f, "us", us)) *us = -1.0;
    if (!tune_double(f, "default_us", def)) *def = -1.0;
    return true;
}

// Run the batch (current schedule) until the GPU has spent >= 25 ms on it:
// its clock needs ~10 ms of continuous work, and candidates timed cold would
// read slow, so that the order of the search would decide the pick.
int warm_batch(sphfilt_batch b, const std::vector<double *> &bufs, hipStream_t s)
{
    double spent = 0.0;
    for (int k = 0; k < 64 && spent < 25000.0; ++k) {
        double us = 0;
        const int rc = time_schedule(b, bufs, s, 4, &us);
        if (rc) return rc;
        spent += 6.0 * kBatchCallsPerRound * us;   // time_schedule runs reps + 2 rounds
    }
    return SPHFILT_OK;
}

int tune(sphfilt_batch b, const char *cache_path)
{
    long long total = 0;
    for (const PatchHost &p : b->patches) total += p.n_points;
    double *scratch = nullptr;
    hipError_t e = hipMalloc((void **)&scratch, sizeof(double) * (size_t)total);
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? SPHFILT_ENOMEM : SPHFILT_EDEVICE;
    std::vector<double *> bufs;
    long long off = 0;
    for (const PatchHost &p : b->patches) {
        bufs.push_back(scratch + off);
        off += p.n_points;
    }
    hipStream_t s = nullptr;
    int rc = SPHFILT_OK;
    if (hipMemset(scratch, 0, sizeof(double) * (size_t)total) != hipSuccess ||
        hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess)
        rc = SPHFILT_EDEVICE;

    // coordinate descent from the untuned schedule: (fused items, split,
    // workgroups per CU), then the theta tile width of each line length, the
    // tiles per theta item, the ring groups per phi item, then split and
    // workgroups per CU again.  The untuned schedule is one of the candidates,
    // so the pick is never slower than it by the tuner's own measurement.
    const Sched start{};
    Sched best = start;
    double best_us = 1e300, default_us = -1.0;
    auto try_sched = [&](const Sched &c) {
        if (rc) return;
        rc = set_sched(b, c);
        double us = 0;
        if (!rc) rc = time_schedule(b, bufs, s, 5, &us);
        if (rc) return;
        if (default_us < 0) default_us = us;          // the first candidate is `start`
        if (us < best_us) {
            best_us = us;
            best = c;
        }
    };
    // warm the GPU up first (see warm_batch)
    if (!rc) rc = warm_batch(b, bufs, s);
    try_sched(start);
    bool any_fused = false;
    for (const PatchHost &p : b->patches) any_fused |= p.tables.n_fused > 0 && p.tables.n_fused == p.tables.theta_active;
    auto split_wpc = [&](int fused) {
        for (int split = 0; split <= 2 && !rc; ++split)
            for (int wpc = -1; wpc <= b->max_wpc && !rc; ++wpc) {
                if (wpc == 0) continue;
                Sched c = best;
                c.fused = fused;
                c.split = split;
                c.wpc = wpc;
                try_sched(c);
            }
    };
    for (int fz = 1; fz >= 0 && !rc; --fz)
        if (fz == 1 || any_fused) split_wpc(fz);
    // theta tile widths, per line length with two-pass theta work
    for (int n : kLines) {
        bool has = false;
        for (const PatchHost &p : b->patches)
            has |= 2 * p.n_theta == n && !(best.fused && p.tables.n_fused > 0 &&
                                           p.tables.n_fused == p.tables.theta_active);
        if (!has) continue;
        const Sched base = best;
        for (int w : {4, 8, 16, 32, 64}) {
            bool valid = false;
            for (const PatchHost &p : b->patches) valid |= 2 * p.n_theta == n && theta_shape_ok(n, w, p.n_phi);
            if (!valid) continue;
            Sched c = base;
            c.cols[n] = w;
            if (c.cols == best.cols) continue;
            try_sched(c);
        }
    }
    for (int t : {2, 4}) {
        Sched c = best;
        c.theta_tiles = t;
        try_sched(c);
    }
    for (int g : {2, 4}) {
        Sched c = best;
        c.phi_groups = g;
        try_sched(c);
    }
    split_wpc(best.fused);

    // confirm: the pick against the untuned schedule, three alternating rounds
    // each; keep the pick only if it is faster by more than 1 %
    if (!rc && !(best.fused == start.fused && best.split == start.split && best.wpc == start.wpc &&
                 best.theta_tiles == start.theta_tiles && best.phi_groups == start.phi_groups &&
                 best.cols == start.cols)) {
        std::vector<double> tb, ts;
        for (int round = 0; round < 3 && !rc; ++round) {
            double us = 0;
            rc = set_sched(b, best);
            if (!rc) rc = time_schedule(b, bufs, s, 5, &us);
            tb.push_back(us);
            if (!rc) rc = set_sched(b, start);
            if (!rc) rc = time_schedule(b, bufs, s, 5, &us);
            ts.push_back(us);
        }
        if (!rc) {
            std::sort(tb.begin(), tb.end());
            std::sort(ts.begin(), ts.end());
            best_us = tb[1];
            default_us = ts[1];
            if (!(tb[1] < 0.99 * ts[1])) {
                best = start;
                best_us = ts[1];
            }
        }
    }

    if (s) (void)hipStreamSynchronize(s);
    // drop the graphs that point at the scratch fields
    for (auto it = b->graphs.begin(); it != b->graphs.end();) {
        if (!it->outs.empty() && it->outs[0] == bufs[0]) {
            free_graph(&*it);
            it = b->graphs.erase(it);
        } else {
            ++it;
        }
    }
    if (s) (void)hipStreamDestroy(s);
    (void)hipFree(scratch);
    if (rc) return rc;
    rc = set_sched(b, best);
    if (rc) return rc;
    b->tuned_us = best_us;
    b->default_us = default_us;
    if (cache_path && !tune_cache_put(cache_path, hex64(b->signature), sched_fields(b, best, best_us, default_us)))
        return SPHFILT_EINVAL;
    return SPHFILT_OK;
}

}  // namespace

extern "C" {

int sphfilt_batch_create(sphfilt_batch *out, int n_patches, const sphfilt_patch_desc *desc,
                         const char *tune_cache_path)
{
    if (!out) return SPHFILT_EINVAL;
    *out = nullptr;
    if (n_patches <= 0 || !desc) return SPHFILT_EINVAL;
    long long shells = 0, th = 0, ph = 0;
    for (int p = 0; p < n_patches; ++p) {
        const sphfilt_patch_desc &d = desc[p];
        const int rc = validate(d.n_r, d.n_theta, d.n_phi, d.n_fields, d.parity, &d.cut);
        if (rc) return rc;
        shells += (long long)d.n_fields * d.n_r;
    }
    if (shells > 0x7fffffffLL) return SPHFILT_EUNSUPPORTED;
    if (fault("alloc")) return SPHFILT_ENOMEM;
    sphfilt_batch b = new (std::nothrow) sphfilt_batch_s();
    if (!b) return SPHFILT_ENOMEM;
    int rc = SPHFILT_OK;
    try {
        std::vector<ThetaItem> all_th;
        std::vector<PhiItem> all_ph;
        std::vector<double> all_fc;
        std::vector<BatchPatchDev> pdev;
        int shell_base = 0;
        for (int p = 0; p < n_patches; ++p) {
            const sphfilt_patch_desc &d = desc[p];
            PatchHost h;
            h.n_r = d.n_r;
            h.n_theta = d.n_theta;
            h.n_phi = d.n_phi;
            h.n_fields = d.n_fields;
            build_items(d.n_r, d.n_theta, d.n_phi, d.n_fields, d.parity, &d.cut, &h.tables);
            h.theta_off = (int)all_th.size();
            h.phi_off = (int)all_ph.size();
            h.shell_base = shell_base;
            h.cols = default_theta_cols(2 * d.n_theta, d.n_phi);
            h.n_points = (long long)d.n_fields * d.n_r * d.n_theta * d.n_phi;
            shell_base += d.n_fields * d.n_r;
            all_th.insert(all_th.end(), h.tables.theta.begin(), h.tables.theta.end());
            all_ph.insert(all_ph.end(), h.tables.phi.begin(), h.tables.phi.end());
            h.phi_rest_off = (int)all_ph.size();
            all_ph.insert(all_ph.end(), h.tables.phi_rest.begin(), h.tables.phi_rest.end());
            h.fc_off = (int)all_fc.size();
            all_fc.insert(all_fc.end(), h.tables.fused_c.begin(), h.tables.fused_c.end());
            b->patches.push_back(std::move(h));
        }
        th = (long long)all_th.size();
        ph = (long long)all_ph.size();
        b->n_shells_total = shell_base;
        hipDeviceProp_t prop;
        if (hipGetDevice(&b->device) != hipSuccess ||
            hipGetDeviceProperties(&prop, b->device) != hipSuccess)
            rc = SPHFILT_EDEVICE;
        if (!rc) {
            b->n_cu = prop.multiProcessorCount;
            b->arch = prop.gcnArchName;
            const size_t colon = b->arch.find(':');
            if (colon != std::string::npos) b->arch.resize(colon);
            bool mixed = false;
            for (int p = 0; p < n_patches; ++p) {
                b->hybrid |= hybrid_args(&desc[p].cut, desc[p].n_fields).present;
                mixed = mixed || mixed_radix_line(2 * desc[p].n_theta) || mixed_radix_line(desc[p].n_phi);
            }
            b->variant = (b->hybrid ? kBatchHybrid : 0) | (mixed ? kBatchMixedRadix : 0);
            b->max_wpc = batch_blocks_per_cu(b->variant);
            b->signature = signature(b->arch, n_patches, desc);
        }
        for (int N : {32, 48, 64, 80, 96, 128, 160, 192, 256}) {
            if (rc) break;
            bool used = false;
            for (const PatchHost &h : b->patches) used |= (2 * h.n_theta == N) || (h.n_phi == N);
            if (!used) continue;
            Twiddle *d = nullptr;
            rc = upload(&d, twiddles(N));
            if (!rc) b->d_tw[N] = d;
        }
        for (int p = 0; p < n_patches && !rc; ++p) {
            const PatchHost &h = b->patches[(size_t)p];
            const HybridArgs ha = hybrid_args(&desc[p].cut, h.n_fields);
            b->hybrid |= ha.present;
            pdev.push_back(BatchPatchDev{b->d_tw[2 * h.n_theta], b->d_tw[h.n_phi], h.n_theta, h.n_phi,
                                         2 * h.n_theta, ilog2_int(h.cols), ha.eps, ha.threshold,
                                         ha.present, 0});
        }
        if (!rc) rc = upload(&b->d_th, all_th);
        if (!rc) rc = upload(&b->d_ph, all_ph);
        if (!rc) rc = upload(&b->d_fc, all_fc);
        if (!rc) rc = upload(&b->d_patches, pdev);
        if (!rc) b->pdev = pdev;
        if (!rc) rc = upload(&b->d_eneg, exp_table());
        if (!rc) rc = upload(&b->d_counters, std::vector<int>((size_t)std::max(1, b->n_shells_total), 0));
        if (!rc) rc = upload(&b->d_tickets, std::vector<int>(3, 0));
        if (!rc) rc = upload(&b->d_error, std::vector<int>(1, 0));
        if (!rc && (hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking) != hipSuccess ||
                    hipStreamCreateWithFlags(&b->side_stream, hipStreamNonBlocking) != hipSuccess ||
                    hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess ||
                    hipEventCreateWithFlags(&b->join, hipEventDisableTiming) != hipSuccess))
            rc = SPHFILT_EDEVICE;
    } catch (const std::bad_alloc &) {
        rc = SPHFILT_ENOMEM;
    }
    (void)th;
    (void)ph;
    // NULL: the cache named by $SPHFILT_TUNE_CACHE, if any
    const char *cache = tune_cache_path ? tune_cache_path : tune_cache_default();
    if (!rc && cache) {
        TuneFields f;
        Sched c;
        double us = -1.0, def = -1.0;
        if (tune_cache_get(cache, hex64(b->signature), &f) && sched_from_fields(b, f, &c, &us, &def)) {
            rc = set_sched(b, c);
            b->tuned_us = us;
            b->default_us = def;
        } else {
            rc = tune(b, cache);
        }
    }
    // the work lists of every mode, and the device address of the static
    // scratch array of the allocation-free entry point (looked up once per
    // device, with the batch's device current)
    // (a failed lookup is retried by the first allocation-free call, which
    // reports it; the other entry points do not need the array)
    if (!rc) rc = ensure_modes(b);
    if (!rc && noalloc_scratch(b->device, &b->noalloc) != hipSuccess) b->noalloc = nullptr;
    if (rc) {
        free_batch(b);
        delete b;
        return rc;
    }
    *out = b;
    return SPHFILT_OK;
}

int sphfilt_batch_destroy(sphfilt_batch batch)
{
    if (!batch) return SPHFILT_OK;
    {
        DeviceGuard g(batch->device);
        (void)hipDeviceSynchronize();
        free_batch(batch);
    }
    delete batch;
    return SPHFILT_OK;
}

int sphfilt_batch_apply(sphfilt_batch batch, const double *const *ins, double *const *outs,
                        int adjoint, void *stream)
{
    if (!batch) return SPHFILT_EINVAL;
    DeviceGuard g(batch->device);
    if (!g.ok) return SPHFILT_EDEVICE;
    return launch(batch, ins, outs, adjoint, (hipStream_t)stream);
}

int sphfilt_batch_apply_noalloc(sphfilt_batch batch, const double *const *ins,
                                double *const *outs, int adjoint, void *stream)
{
    if (!batch) return SPHFILT_EINVAL;
    DeviceGuard g(batch->device);
    if (!g.ok) return SPHFILT_EDEVICE;
    return launch_noalloc(batch, ins, outs, adjoint, (hipStream_t)stream);
}

int sphfilt_batch_tune(sphfilt_batch batch, const char *tune_cache_path)
{
    if (!batch) return SPHFILT_EINVAL;
    DeviceGuard g(batch->device);
    if (!g.ok) return SPHFILT_EDEVICE;
    return tune(batch, tune_cache_path);
}

int sphfilt_batch_set_schedule(sphfilt_batch batch, int split, int workgroups_per_cu)
{
    if (!batch || split < 0 || split > 2 || workgroups_per_cu < -1 ||
        workgroups_per_cu > batch->max_wpc)
        return SPHFILT_EINVAL;
    batch->split = split;
    batch->wpc = workgroups_per_cu;
    return SPHFILT_OK;
}

int sphfilt_batch_get_schedule(sphfilt_batch batch, int *split, int *workgroups_per_cu,
                               double *tuned_us)
{
    if (!batch) return SPHFILT_EINVAL;
    if (split) *split = batch->split;
    if (workgroups_per_cu) *workgroups_per_cu = effective_wpc(batch, batch->wpc);
    if (tuned_us) *tuned_us = batch->tuned_us;
    return SPHFILT_OK;
}

int sphfilt_batch_set_schedule_ex(sphfilt_batch batch, const sphfilt_batch_schedule *sched)
{
    if (!batch || !sched) return SPHFILT_EINVAL;
    const sphfilt_batch_schedule &q = *sched;
    auto pow2_le8 = [](int v) { return v == 1 || v == 2 || v == 4 || v == 8; };
    if (q.split < 0 || q.split > 2 || q.workgroups_per_cu < -1 || q.workgroups_per_cu > batch->max_wpc ||
        (q.fused != 0 && q.fused != 1) || !pow2_le8(q.theta_tiles) || !pow2_le8(q.phi_groups))
        return SPHFILT_EINVAL;
    Sched c;
    c.split = q.split;
    c.wpc = q.workgroups_per_cu;
    c.fused = q.fused;
    c.theta_tiles = q.theta_tiles;
    c.phi_groups = q.phi_groups;
    for (int i = 0; i < 9; ++i) {
        const int w = q.theta_cols[i];
        if (w == 0) continue;
        if (w != 4 && w != 8 && w != 16 && w != 32 && w != 64) return SPHFILT_EINVAL;
        c.cols[kLines[i]] = w;
    }
    DeviceGuard g(batch->device);
    if (!g.ok) return SPHFILT_EDEVICE;
    return set_sched(batch, c);
}

int sphfilt_batch_get_schedule_ex(sphfilt_batch batch, sphfilt_batch_schedule *sched)
{
    if (!batch || !sched) return SPHFILT_EINVAL;
    sphfilt_batch_schedule q{};
    q.split = batch->split;
    q.workgroups_per_cu = effective_wpc(batch, batch->wpc);
    q.fused = batch->fused;
    q.theta_tiles = batch->theta_tiles;
    q.phi_groups = batch->phi_groups;
    for (int i = 0; i < 9; ++i) {
        auto it = batch->theta_cols.find(kLines[i]);
        q.theta_cols[i] = it == batch->theta_cols.end() ? 0 : it->second;
    }
    q.tuned_us = batch->tuned_us;
    q.default_us = batch->default_us;
    *sched = q;
    return SPHFILT_OK;
}

int sphfilt_batch_status(sphfilt_batch batch, int *device_error)
{
    if (!batch || !device_error) return SPHFILT_EINVAL;
    DeviceGuard g(batch->device);
    if (!g.ok) return SPHFILT_EDEVICE;
    if (hipDeviceSynchronize() != hipSuccess) return SPHFILT_EDEVICE;
    // the error word of the last call: the batch's own, or the static array's
    // after an allocation-free call (valid until another such call on the device)
    const int *word = batch->last_noalloc && batch->noalloc
                          ? reinterpret_cast<const int *>(batch->noalloc) + 3
                          : batch->d_error;
    if (hipMemcpy(device_error, word, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
        return SPHFILT_EDEVICE;
    return SPHFILT_OK;
}

int sphfilt_batch_stats(sphfilt_batch batch, sphfilt_stats *out)
{
    if (!batch || !out) return SPHFILT_EINVAL;
    std::memset(out, 0, sizeof(*out));
    for (const PatchHost &p : batch->patches) {
        sphfilt_stats s;
        fill_stats(p.n_r, p.n_theta, p.n_phi, p.n_fields, p.tables, &s);
        long long *dst = (long long *)out;
        const long long *src = (const long long *)&s;
        for (size_t i = 0; i < sizeof(s) / sizeof(long long); ++i) dst[i] += src[i];
    }
    if (!batch->fused) {
        out->shells_fused = 0;
        out->bytes_fused_inplace = out->bytes_forward_inplace;
    }
    return SPHFILT_OK;
}

int sphfilt_batch_set_fused(sphfilt_batch batch, int enable)
{
    if (!batch || (enable != 0 && enable != 1)) return SPHFILT_EINVAL;
    if (batch->fused == enable) return SPHFILT_OK;
    DeviceGuard g(batch->device);
    if (!g.ok) return SPHFILT_EDEVICE;
    if (hipDeviceSynchronize() != hipSuccess) return SPHFILT_EDEVICE;
    free_work(batch);
    batch->fused = enable;
    return ensure_modes(batch);
}

int sphfilt_batch_get_fused(sphfilt_batch batch, int *enable, int *shells_fused)
{
    if (!batch) return SPHFILT_EINVAL;
    int n = 0;
    for (const PatchHost &p : batch->patches)
        if (patch_fused(batch, p)) n += p.tables.n_fused;
    if (enable) *enable = batch->fused;
    if (shells_fused) *shells_fused = n;
    return SPHFILT_OK;
}

}  // extern "C"
