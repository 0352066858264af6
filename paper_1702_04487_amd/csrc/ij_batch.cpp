// ij_batch.cpp -- batches of independent lattices (parameter sweeps) stepped
// together: one launch per kind of step work covers every case, the steps
// between diagnostics samples replay as one captured graph, and the tile
// shape is chosen by timing candidates on the batch itself.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "ij_internal.h"

using namespace ij_host;

namespace {

thread_local std::string g_batch_create_error;

// tile shapes the autotuner times: waves across x, rows per workgroup, and
// whether the columns past the last full strip go to 64-column strips; each
// with persistent workgroups and with one workgroup per tile
const int kCandidates[][3] = {{1, 32, 0}, {2, 32, 0}, {2, 64, 0}, {4, 32, 0}, {4, 64, 0}, {2, 64, 1}, {4, 64, 1},
                              {1, 1, 0},  {2, 1, 0},  {4, 1, 0}};

// autotuned shapes by batch signature (lattice sizes, walls and diagnostics
// interval of every case), for the life of the process
std::mutex g_tune_mutex;
struct Tiling {
    int waves_x, rows, mixed, persistent;
};
std::map<std::vector<int64_t>, Tiling> g_tune_cache;

}  // namespace

struct ij_batch {
    std::vector<ij_sim*> sims;
    int waves_x = 4, rows_per_block = 1, mixed = 0, persistent = 1;
    int64_t t = 0;
    int64_t diag_every = 0;
    int graph_steps = 0;   // steps per captured graph, 0: plain launches
    // device tables: (case, strip, row block) tiles of the wide and the
    // 64-column tail strips, plain and general, in one allocation
    ij::CaseRec* d_cases = nullptr;
    int4* d_tiles = nullptr;
    size_t cap_tiles = 0;
    std::vector<int4> tiles_host;   // wide | tail | general wide | general tail
    ij::BatchTiles T{};
    int64_t* d_t = nullptr;
    int64_t* d_nrec = nullptr;
    int* d_active = nullptr;
    // pinned staging of the per-call uploads
    ij::CaseRec* h_cases = nullptr;
    int64_t* h_nrec = nullptr;
    int* h_active = nullptr;
    hipEvent_t staged = nullptr;   // the uploads of the last call have been read
    int max_nx = 0, max_ny = 0;
    size_t max_parts = 0;   // sample partials of the widest case, [ceil(nx/64)][ny]
    // graph of graph_steps steps starting at a step that is a multiple of it
    hipStream_t cs = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    // the general pieces run beside the row launch on a second stream
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    int graph_len = 0;
    std::string err;
};

namespace {

ij_status bfail(ij_batch* b, ij_status st, const std::string& m)
{
    if (b)
        b->err = m;
    else
        g_batch_create_error = m;
    return st;
}

ij_status bhip(ij_batch* b, hipError_t e, const char* where)
{
    return bfail(b, IJ_ERR_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

#define IJB_HIP(b, call)                                     \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return bhip(b, e_, #call);     \
    } while (0)

void drop_graph(ij_batch* b)
{
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->gexec = nullptr;
    b->graph = nullptr;
    b->graph_len = 0;
}

int64_t lcm64(int64_t a, int64_t b)
{
    int64_t x = a, y = b;
    while (y) {
        const int64_t r = x % y;
        x = y;
        y = r;
    }
    return a / x * b;
}

// steps per graph: a multiple of 2 (buffer parity) and of the diagnostics
// interval, close to the requested count
int64_t graph_period(const ij_batch* b)
{
    const int64_t unit = b->diag_every > 0 ? lcm64(2, b->diag_every) : 2;
    const int64_t want = std::max<int64_t>(b->graph_steps, 1);
    return (want + unit - 1) / unit * unit;
}

// workgroups of the two plain launches: as many as are resident at once
// (each running a contiguous run of tiles), or one per tile
ij_status set_grids(ij_batch* b)
{
    ij::BatchTiles& T = b->T;
    int gw = T.n_wide, gt = T.n_tail;
    if (b->persistent) {
        gw = ij::batch_resident_workgroups(b->waves_x);
        gt = ij::batch_resident_workgroups(1);
        if (gw <= 0 || gt <= 0) return bfail(b, IJ_ERR_DEVICE, "occupancy query failed");
    }
    if (gw != T.grid_wide || gt != T.grid_tail) drop_graph(b);
    T.grid_wide = gw;
    T.grid_tail = gt;
    return IJ_OK;
}

// tile lists of the launches from the members' current tilings
ij_status build_tiles(ij_batch* b)
{
    std::vector<int4> lists[4];   // wide, tail, general, rows
    for (size_t c = 0; c < b->sims.size(); ++c) {
        const ij_sim* s = b->sims[c];
        if (b->rows_per_block == 1) {
            // pieces of 64 columns of every plain (row, strip) of the case, row-major
            for (int y = 0; y < s->ny; ++y)
                for (int k = 0; k < s->n_strips; ++k) {
                    if (!s->plain_host[(size_t)k * s->ny + y]) continue;
                    const int x1 = k + 1 < s->n_strips ? s->strip_x0[(size_t)k + 1] : s->nx;
                    for (int x = s->strip_x0[(size_t)k]; x < x1; x += 64)
                        lists[3].push_back(make_int4((int)c, y, x, std::min(64, x1 - x)));
                }
        } else
        // plain tiles that hold a plain row (a block of rows that all sit
        // beside solid nodes, such as a nozzle channel, is the general
        // launch's alone)
        for (int rb = 0; rb < s->n_rb; ++rb)
            for (int k = 0; k < s->n_strips; ++k)
                if (s->tile_plain[(size_t)rb * s->n_strips + k]) {
                    const int y0 = rb * s->rows_per_block, h = std::min(s->ny - y0, s->rows_per_block);
                    // bit 30: an odd row block (it may walk its rows downwards)
                    lists[k < s->n_wide ? 0 : 1].push_back(
                        make_int4((int)c, k, y0 | (h << 16) | ((rb & 1) << 30), s->strip_x0[(size_t)k]));
                }
        for (const int4& g : s->gtiles_host) lists[2].push_back(make_int4((int)c, g.x, g.y | (g.w << 16), g.z));
    }
    std::vector<int4> all;
    for (auto& l : lists) all.insert(all.end(), l.begin(), l.end());
    const int counts[4] = {(int)lists[0].size(), (int)lists[1].size(), (int)lists[2].size(), (int)lists[3].size()};
    const bool same = all.size() == b->tiles_host.size() &&
                      std::memcmp(all.data(), b->tiles_host.data(), all.size() * sizeof(int4)) == 0 &&
                      counts[0] == b->T.n_wide && counts[1] == b->T.n_tail && counts[2] == b->T.n_gen &&
                      counts[3] == b->T.n_rows;
    if (same && (b->d_tiles || all.empty())) return set_grids(b);
    if (all.size() > b->cap_tiles) {
        if (b->d_tiles) (void)hipFree(b->d_tiles);
        b->d_tiles = nullptr;
        b->cap_tiles = 0;
        if (hipMalloc(&b->d_tiles, all.size() * sizeof(int4)) != hipSuccess)
            return bfail(b, IJ_ERR_OOM, "tile list allocation failed");
        b->cap_tiles = all.size();
    }
    if (!all.empty()) IJB_HIP(b, hipMemcpy(b->d_tiles, all.data(), all.size() * sizeof(int4), hipMemcpyHostToDevice));
    b->tiles_host.swap(all);
    ij::BatchTiles& T = b->T;
    T.wide = b->d_tiles;
    T.tail = T.wide + counts[0];
    T.gen = T.tail + counts[1];
    T.rows = T.gen + counts[2];
    T.n_wide = counts[0];
    T.n_tail = counts[1];
    T.n_gen = counts[2];
    T.n_rows = counts[3];
    drop_graph(b);
    return set_grids(b);
}

// Cases the device switched off since the host last looked are learnt from
// their samples (which also tells which of a case's buffers holds its frozen
// state).  Synchronises the stream.
ij_status learn_frozen(ij_batch* b, hipStream_t st)
{
    IJB_HIP(b, hipEventSynchronize(b->staged));   // the previous uploads have been read
    const size_t nc = b->sims.size();
    IJB_HIP(b, hipStreamSynchronize(st));
    IJB_HIP(b, hipMemcpy(b->h_active, b->d_active, nc * sizeof(int), hipMemcpyDeviceToHost));
    for (size_t c = 0; c < nc; ++c) {
        ij_sim* s = b->sims[c];
        if (!b->h_active[c] && s->unstable_step < 0 && drain_samples(s, st) != IJ_OK)
            return bfail(b, IJ_ERR_DEVICE, s->err);
    }
    return IJ_OK;
}

// Case records, sample counters and guard flags of the current state, on
// the stream.  Relative parity 0 is each case's current buffer.
ij_status stage(ij_batch* b, hipStream_t st)
{
    const ij_status fr = learn_frozen(b, st);
    if (fr != IJ_OK) return fr;
    for (size_t c = 0; c < b->sims.size(); ++c) {
        ij_sim* s = b->sims[c];
        ij::CaseRec& r = b->h_cases[c];
        std::memset(&r, 0, sizeof r);
        r.P = s->K;
        r.buf[0] = s->buf[s->cur];
        r.buf[1] = s->buf[1 - s->cur];
        r.wall = s->wall;
        r.plain = s->plain;
        r.parts = s->sample_parts;
        r.rows = s->rows;
        r.ring = s->samples;
        r.row0 = (int)s->p.diag_row0;
        r.a_min = (int)std::ceil(4.0 * s->p.width * s->p.width);
        r.band = diag_band(s->p.width);
        r.t_pos = s->p.t_pos;
        r.t_neg = s->p.t_neg;
        r.t_idle = s->p.t_idle;
        r.periodic = (int)s->p.periodic_pulse;
        r.f_pos = s->p.f_pos;
        r.f_neg = s->p.f_neg;
        r.u_limit = u_limit(s->p);
        b->h_nrec[c] = s->n_dev_samples;
        b->h_active[c] = s->unstable_step < 0 ? 1 : 0;
    }
    const size_t n = b->sims.size();
    IJB_HIP(b, hipMemcpyAsync(b->d_cases, b->h_cases, n * sizeof(ij::CaseRec), hipMemcpyHostToDevice, st));
    IJB_HIP(b, hipMemcpyAsync(b->d_nrec, b->h_nrec, n * sizeof(int64_t), hipMemcpyHostToDevice, st));
    IJB_HIP(b, hipMemcpyAsync(b->d_active, b->h_active, n * sizeof(int), hipMemcpyHostToDevice, st));
    IJB_HIP(b, hipEventRecord(b->staged, st));
    IJB_HIP(b, ij::launch_batch_set_time(b->d_t, b->t, b->d_cases, (int)b->sims.size(), st));
    return IJ_OK;
}

// One step at relative parity `parity` on stream st; a diagnostics sample
// first when `diag`.
hipError_t one_step(ij_batch* b, int parity, bool diag, bool with_tick, hipStream_t st)
{
    hipError_t e = hipSuccess;
    if (diag) e = ij::launch_batch_sample_begin(b->d_cases, (int)b->sims.size(), b->max_parts, st);
    if (e == hipSuccess && b->T.n_rows > 0 && b->T.n_gen > 0) {
        // the row pieces and the general pieces touch disjoint rows: the
        // latency-bound pieces run on the side stream beside the row launch
        e = hipEventRecord(b->ev_fork, st);
        if (e == hipSuccess) e = hipStreamWaitEvent(b->side, b->ev_fork, 0);
        if (e == hipSuccess)
            e = ij::launch_batch_general(b->T, b->d_cases, parity, b->d_active, b->waves_x, diag, b->side);
        if (e == hipSuccess) e = ij::launch_batch_rows(b->T, b->d_cases, parity, b->d_active, b->waves_x, diag, st);
        if (e == hipSuccess) e = hipEventRecord(b->ev_join, b->side);
        if (e == hipSuccess) e = hipStreamWaitEvent(st, b->ev_join, 0);
    } else if (e == hipSuccess) {
        e = ij::launch_batch_collide(b->T, b->d_cases, parity, b->d_active, b->waves_x, diag, st);
    }
    if (e == hipSuccess && diag)
        e = ij::launch_batch_sample_end(b->d_cases, (int)b->sims.size(), b->max_ny, b->d_t, b->d_nrec, b->d_active, st);
    if (e == hipSuccess && with_tick)
        e = ij::launch_batch_tick(b->d_t, b->d_cases, (int)b->sims.size(), b->d_active, st);
    return e;
}

ij_status capture_graph(ij_batch* b, int64_t len)
{
    drop_graph(b);
    IJB_HIP(b, hipStreamBeginCapture(b->cs, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int64_t j = 0; j < len && e == hipSuccess; ++j)
        e = one_step(b, (int)(j & 1), b->diag_every > 0 && j % b->diag_every == 0, true, b->cs);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(b->cs, &g);
    if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return bhip(b, e, "graph capture");
    }
    if (e2 != hipSuccess) return bhip(b, e2, "hipStreamEndCapture");
    b->graph = g;
    IJB_HIP(b, hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0));
    b->graph_len = (int)len;
    return IJ_OK;
}

// samples a run of n steps from step t records at interval k
int64_t samples_in(int64_t t, int64_t n, int64_t k)
{
    if (k <= 0 || n <= 0) return 0;
    const int64_t first = (t + k - 1) / k * k;
    return first >= t + n ? 0 : (t + n - 1 - first) / k + 1;
}

ij_status check_members(ij_batch* b)
{
    bool all_zero = true, all_same = true;
    for (const ij_sim* s : b->sims) {
        if (!s->initialised) return bfail(b, IJ_ERR_STATE, "every case must be initialised before stepping");
        all_zero = all_zero && s->t == 0;
        all_same = all_same && s->t == b->t;
    }
    if (all_zero) b->t = 0;
    else if (!all_same) return bfail(b, IJ_ERR_STATE, "cases are at different steps (re-initialise all of them)");
    return IJ_OK;
}

// n steps; diagnostics and the members' bookkeeping follow the single-case
// ij_step exactly.
ij_status run_steps(ij_batch* b, int64_t n, hipStream_t st, bool use_graph)
{
    if (n <= 0) return IJ_OK;
    ij_status r = stage(b, st);
    if (r != IJ_OK) return r;
    int64_t j = 0;
    const int64_t period = use_graph ? graph_period(b) : 0;
    bool on_cs = false;
    while (j < n) {
        const int64_t tj = b->t + j;
        if (period > 0 && tj % period == 0 && (j & 1) == 0 && n - j >= period) {
            if (!b->gexec || b->graph_len != period) {   // tile changes drop the graph
                r = capture_graph(b, period);
                if (r != IJ_OK) return r;
            }
            if (!on_cs) {
                IJB_HIP(b, hipEventRecord(b->ev_in, st));
                IJB_HIP(b, hipStreamWaitEvent(b->cs, b->ev_in, 0));
                on_cs = true;
            }
            IJB_HIP(b, hipGraphLaunch(b->gexec, b->cs));
            j += period;
            continue;
        }
        if (on_cs) {
            IJB_HIP(b, hipEventRecord(b->ev_out, b->cs));
            IJB_HIP(b, hipStreamWaitEvent(st, b->ev_out, 0));
            on_cs = false;
        }
        const hipError_t e = one_step(b, (int)(j & 1), b->diag_every > 0 && tj % b->diag_every == 0, true, st);
        if (e != hipSuccess) return bhip(b, e, "batched step kernels");
        ++j;
    }
    if (on_cs) {
        IJB_HIP(b, hipEventRecord(b->ev_out, b->cs));
        IJB_HIP(b, hipStreamWaitEvent(st, b->ev_out, 0));
    }
    const int64_t ns = samples_in(b->t, n, b->diag_every);
    for (ij_sim* s : b->sims) {
        s->t = b->t + n;
        // a case switched off before this call keeps its buffer (the device
        // swaps its two buffers after every step instead)
        if ((n & 1) && s->unstable_step < 0) s->cur = 1 - s->cur;
        s->n_dev_samples += ns;
    }
    b->t += n;
    return IJ_OK;
}

std::vector<int64_t> signature(const ij_batch* b)
{
    std::vector<int64_t> sig;
    sig.push_back((int64_t)b->sims.size());
    for (const ij_sim* s : b->sims) {
        sig.push_back(s->nx);
        sig.push_back(s->ny);
        sig.push_back(s->p.bc_y);
        uint64_t h = 1469598103934665603ull;   // FNV-1a of the wall mask
        for (uint8_t v : s->wall_host) h = (h ^ v) * 1099511628211ull;
        sig.push_back((int64_t)h);
    }
    return sig;
}

ij_status apply_tiling(ij_batch* b, int waves_x, int rows, int mixed, int persistent)
{
    if (rows == 1) mixed = 0;   // a row tile's waves run to the case's edge: no tail strips
    for (ij_sim* s : b->sims) {
        s->waves_x = waves_x;
        s->rows_per_block = rows;
        s->mixed_strips = mixed != 0;
        if (build_plain(s) != IJ_OK) return bfail(b, IJ_ERR_DEVICE, s->err);
    }
    b->waves_x = waves_x;
    b->rows_per_block = rows;
    b->mixed = mixed != 0;
    b->persistent = persistent != 0;
    return build_tiles(b);
}

}  // namespace

extern "C" {

ij_status ij_batch_create(const ij_params* cases, int32_t n, ij_batch** out)
{
    if (!out) return bfail(nullptr, IJ_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!cases || n <= 0) return bfail(nullptr, IJ_ERR_INVALID_ARG, "need at least one case");
    if (n > 65535) return bfail(nullptr, IJ_ERR_INVALID_ARG, "at most 65535 cases");
    for (int32_t c = 0; c < n; ++c) {
        const std::string v = validate(cases[c]);
        if (!v.empty()) return bfail(nullptr, IJ_ERR_INVALID_ARG, "case " + std::to_string(c) + ": " + v);
        if (cases[c].diag_every != cases[0].diag_every)
            return bfail(nullptr, IJ_ERR_INVALID_ARG, "every case must have the same diag_every");
    }
    ij_batch* b = new ij_batch();
    auto cleanup = [&](ij_status st, const std::string& m) {
        const std::string msg = m;
        ij_batch_destroy(b);
        return bfail(nullptr, st, msg);
    };
    b->diag_every = cases[0].diag_every;
    for (int32_t c = 0; c < n; ++c) {
        ij_sim* s = nullptr;
        const ij_status r = ij_create(&cases[c], &s);
        if (r != IJ_OK) return cleanup(r, "case " + std::to_string(c) + ": " + ij_last_error(nullptr));
        s->in_batch = true;
        b->sims.push_back(s);
        b->max_nx = std::max(b->max_nx, s->nx);
        b->max_ny = std::max(b->max_ny, s->ny);
        // the partials a sampling step reduces (each case's sample is taken
        // inside the collide launches)
        const size_t np = (size_t)((s->nx + 63) / 64) * (size_t)s->ny;
        b->max_parts = std::max(b->max_parts, np);
        if (hipMalloc(&s->sample_parts, np * sizeof(ij::DiagRow)) != hipSuccess) {
            s->sample_parts = nullptr;
            return cleanup(IJ_ERR_OOM, "case " + std::to_string(c) + ": sample partials allocation failed");
        }
    }
    const size_t nb = (size_t)n;
    if (hipMalloc(&b->d_cases, nb * sizeof(ij::CaseRec)) != hipSuccess ||
        hipMalloc(&b->d_t, sizeof(int64_t)) != hipSuccess || hipMalloc(&b->d_nrec, nb * sizeof(int64_t)) != hipSuccess ||
        hipMalloc(&b->d_active, nb * sizeof(int)) != hipSuccess ||
        hipMemset(b->d_active, 0, nb * sizeof(int)) != hipSuccess ||
        hipHostMalloc(&b->h_cases, nb * sizeof(ij::CaseRec), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(&b->h_nrec, nb * sizeof(int64_t), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(&b->h_active, nb * sizeof(int), hipHostMallocDefault) != hipSuccess)
        return cleanup(IJ_ERR_OOM, "batch table allocation failed");
    if (hipStreamCreateWithFlags(&b->cs, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->staged, hipEventDisableTiming) != hipSuccess)
        return cleanup(IJ_ERR_DEVICE, "stream or event creation failed");
    const ij_status r = apply_tiling(b, b->waves_x, b->rows_per_block, b->mixed, b->persistent);
    if (r != IJ_OK) return cleanup(r, b->err);
    *out = b;
    return IJ_OK;
}

void ij_batch_destroy(ij_batch* b)
{
    if (!b) return;
    // steps without graphs run on the caller's stream: wait for the whole
    // device, not only for the batch's own streams, before freeing
    (void)hipDeviceSynchronize();
    drop_graph(b);
    for (ij_sim* s : b->sims) destroy_sim(s);
    if (b->d_cases) (void)hipFree(b->d_cases);
    if (b->d_tiles) (void)hipFree(b->d_tiles);
    if (b->d_t) (void)hipFree(b->d_t);
    if (b->d_nrec) (void)hipFree(b->d_nrec);
    if (b->d_active) (void)hipFree(b->d_active);
    if (b->staged) (void)hipEventSynchronize(b->staged);
    if (b->h_cases) (void)hipHostFree(b->h_cases);
    if (b->h_nrec) (void)hipHostFree(b->h_nrec);
    if (b->h_active) (void)hipHostFree(b->h_active);
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_out) (void)hipEventDestroy(b->ev_out);
    if (b->staged) (void)hipEventDestroy(b->staged);
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    if (b->ev_join) (void)hipEventDestroy(b->ev_join);
    if (b->side) (void)hipStreamDestroy(b->side);
    if (b->cs) (void)hipStreamDestroy(b->cs);
    delete b;
}

const char* ij_batch_last_error(const ij_batch* b) { return b ? b->err.c_str() : g_batch_create_error.c_str(); }

int32_t ij_batch_size(const ij_batch* b) { return b ? (int32_t)b->sims.size() : -1; }

ij_status ij_batch_case(ij_batch* b, int32_t i, ij_sim** out)
{
    if (!b || !out) return IJ_ERR_INVALID_ARG;
    if (i < 0 || i >= (int32_t)b->sims.size()) return bfail(b, IJ_ERR_INVALID_ARG, "case index out of range");
    *out = b->sims[(size_t)i];
    return IJ_OK;
}

int64_t ij_batch_time(const ij_batch* b) { return b ? b->t : -1; }

ij_status ij_batch_set_graph(ij_batch* b, int32_t steps_per_graph)
{
    if (!b) return IJ_ERR_INVALID_ARG;
    if (steps_per_graph < 0 || steps_per_graph > 100000)
        return bfail(b, IJ_ERR_INVALID_ARG, "steps_per_graph must lie in [0, 100000]");
    b->graph_steps = steps_per_graph;
    drop_graph(b);
    return IJ_OK;
}

ij_status ij_batch_set_tiling(ij_batch* b, int32_t waves_x, int32_t rows_per_block, int32_t mixed_strips,
                              int32_t persistent)
{
    if (!b) return IJ_ERR_INVALID_ARG;
    if (waves_x != 1 && waves_x != 2 && waves_x != 4) return bfail(b, IJ_ERR_INVALID_ARG, "waves_x must be 1, 2 or 4");
    if (rows_per_block < 1 || rows_per_block > 1024)
        return bfail(b, IJ_ERR_INVALID_ARG, "rows_per_block must lie in [1, 1024]");
    return apply_tiling(b, waves_x, rows_per_block, mixed_strips != 0, persistent != 0);
}

ij_status ij_batch_get_tiling(const ij_batch* b, int32_t* waves_x, int32_t* rows_per_block, int32_t* mixed_strips,
                              int32_t* persistent)
{
    if (!b) return IJ_ERR_INVALID_ARG;
    if (waves_x) *waves_x = b->waves_x;
    if (rows_per_block) *rows_per_block = b->rows_per_block;
    if (mixed_strips) *mixed_strips = b->mixed;
    if (persistent) *persistent = b->persistent;
    return IJ_OK;
}

ij_status ij_batch_step(ij_batch* b, int64_t nsteps, void* stream)
{
    if (!b) return IJ_ERR_INVALID_ARG;
    if (nsteps < 0) return bfail(b, IJ_ERR_INVALID_ARG, "nsteps < 0");
    ij_status r = check_members(b);
    if (r == IJ_OK) r = build_tiles(b);   // a member's wall may have changed its tiles
    if (r != IJ_OK) return r;
    hipStream_t st = (hipStream_t)stream;
    int64_t done = 0;
    while (done < nsteps) {
        // keep every member's sample ring within its capacity
        int64_t room = kSampleCap;
        for (const ij_sim* s : b->sims) room = std::min(room, kSampleCap - s->n_dev_samples);
        int64_t chunk = nsteps - done;
        const int64_t k = b->diag_every;
        if (k > 0 && samples_in(b->t, chunk, k) > room) {
            if (room <= 0) {
                for (ij_sim* s : b->sims)
                    if (drain_samples(s, st) != IJ_OK) return bfail(b, IJ_ERR_DEVICE, s->err);
                continue;
            }
            // up to, not including, the step of sample number room + 1
            const int64_t first = (b->t + k - 1) / k * k;
            chunk = first + room * k - b->t;
        }
        r = run_steps(b, chunk, st, b->graph_steps > 0);
        if (r != IJ_OK) return r;
        done += chunk;
    }
    return IJ_OK;
}

ij_status ij_batch_autotune(ij_batch* b, int32_t trial_steps, void* stream, int32_t* waves_x, int32_t* rows_per_block,
                            int32_t* mixed_strips, int32_t* persistent, double* ms_per_step)
{
    if (!b) return IJ_ERR_INVALID_ARG;
    if (trial_steps < 2 || trial_steps > 10000) return bfail(b, IJ_ERR_INVALID_ARG, "trial_steps must lie in [2, 10000]");
    ij_status r = check_members(b);
    if (r != IJ_OK) return r;
    hipStream_t st = (hipStream_t)stream;
    const std::vector<int64_t> sig = signature(b);
    {
        std::lock_guard<std::mutex> lk(g_tune_mutex);
        auto it = g_tune_cache.find(sig);
        if (it != g_tune_cache.end()) {
            r = apply_tiling(b, it->second.waves_x, it->second.rows, it->second.mixed, it->second.persistent);
            if (r != IJ_OK) return r;
            if (waves_x) *waves_x = b->waves_x;
            if (rows_per_block) *rows_per_block = b->rows_per_block;
            if (mixed_strips) *mixed_strips = b->mixed;
            if (persistent) *persistent = b->persistent;
            if (ms_per_step) *ms_per_step = -1.0;   // from the cache, not timed
            return IJ_OK;
        }
    }
    // keep the state: trial steps run on the live buffers and are undone
    r = learn_frozen(b, st);   // each case's current buffer
    if (r != IJ_OK) return r;
    std::vector<void*> saved(b->sims.size(), nullptr);
    auto release = [&]() {
        (void)hipStreamSynchronize(st);
        for (void* p : saved)
            if (p) (void)hipFree(p);
    };
    for (size_t c = 0; c < b->sims.size(); ++c) {
        ij_sim* s = b->sims[c];
        const size_t bytes = buffer_bytes(s->plane);
        if (hipMalloc(&saved[c], bytes) != hipSuccess) {
            release();
            return bfail(b, IJ_ERR_OOM, "autotune snapshot allocation failed");
        }
        if (hipMemcpyAsync(saved[c], s->buf[s->cur], bytes, hipMemcpyDeviceToDevice, st) != hipSuccess) {
            release();
            return bfail(b, IJ_ERR_DEVICE, "autotune snapshot copy failed");
        }
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        release();
        return bfail(b, IJ_ERR_DEVICE, "event creation failed");
    }
    const int old_w = b->waves_x, old_r = b->rows_per_block, old_m = b->mixed, old_p = b->persistent;
    double best = 1e300;
    int bw = old_w, br = old_r, bm = old_m, bp = old_p;
    trial_steps += trial_steps & 1;   // even: every trial ends on the buffer it started from
    for (int trial = 0; trial < 2 * (int)(sizeof kCandidates / sizeof kCandidates[0]); ++trial) {
        const int* cand = kCandidates[trial >> 1];
        const int pers = trial & 1;
        r = apply_tiling(b, cand[0], cand[1], cand[2], pers);
        if (r == IJ_OK) r = stage(b, st);   // the tables of the new tiling
        if (r != IJ_OK) break;
        // two untimed steps, then the timed ones (no diagnostics: the tile
        // shape does not change them)
        hipError_t e = hipSuccess;
        for (int j = 0; j < 2 && e == hipSuccess; ++j) e = one_step(b, j & 1, false, false, st);
        if (e == hipSuccess) e = hipEventRecord(e0, st);
        for (int j = 0; j < trial_steps && e == hipSuccess; ++j) e = one_step(b, j & 1, false, false, st);
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
            r = bhip(b, e, "autotune trial");
            break;
        }
        const double per = ms / trial_steps;
        if (per < best) {
            best = per;
            bw = cand[0];
            br = cand[1];
            bm = cand[2];
            bp = pers;
        }
    }
    // restore the state whatever happened
    for (size_t c = 0; c < b->sims.size(); ++c) {
        ij_sim* s = b->sims[c];
        (void)hipMemcpyAsync(s->buf[s->cur], saved[c], buffer_bytes(s->plane), hipMemcpyDeviceToDevice, st);
    }
    release();
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (r != IJ_OK) {
        (void)apply_tiling(b, old_w, old_r, old_m, old_p);
        return r;
    }
    r = apply_tiling(b, bw, br, bm, bp);
    if (r != IJ_OK) return r;
    {
        std::lock_guard<std::mutex> lk(g_tune_mutex);
        g_tune_cache[sig] = {bw, br, bm, bp};
    }
    if (waves_x) *waves_x = bw;
    if (rows_per_block) *rows_per_block = br;
    if (mixed_strips) *mixed_strips = bm;
    if (persistent) *persistent = bp;
    if (ms_per_step) *ms_per_step = best;
    return IJ_OK;
}

}  // extern "C"
