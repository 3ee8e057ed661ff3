// Ensemble of independent simulations advanced by one persistent launch per
// step (include/lbch_batch.h).
#include "../../include/lbch_batch.h"
#include "lbch_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

using namespace lbch;

#define HIP_TRY(expr)                                                                                    \
    do {                                                                                                 \
        hipError_t e_ = (expr);                                                                          \
        if (e_ != hipSuccess) return fail(LBCH_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

namespace {

constexpr int kGraphLaunches = 16;   // launches per captured graph (even: buffer parity preserved)

// Launch configuration of one depth (time steps per launch): descriptors, the
// tile -> member list and the persistent grid.
struct BatchConfig {
    int nt = 128, hc_user = 0, blocks_user = 0;
    int hc = 0;                      // chunk height in use (hc_user, or the default for the ensemble)
    int total_tiles = 0, nblocks = 0;
    void* d_members = nullptr;       // BatchMember<T>[count]
    int* d_tile_member = nullptr;    // int[total_tiles]
};

struct Member {
    lbch_params p;
    Grid g;
    long long base;
    RedCoef rc;
    StepCoef<double> cd;
    StepCoef<float> cf;
    bool initialized;
};

}  // namespace

struct lbch_batch {
    int precision = 0;
    size_t esize = 8;
    std::vector<Member> m;
    void* f[2] = {nullptr, nullptr};
    int cur = 0;
    hipStream_t stream = nullptr;
    int64_t step = 0;
    long long total_elems = 0;
    // tiling
    int depth = 2;                   // time steps per launch (odd remainders use depth 1)
    BatchConfig cfg[2];              // index depth - 1
    bool unit_all = true;
    unsigned long long* d_counter = nullptr;   // work-queue counters, one per depth
    bool counter_dirty = true;
    // reductions
    double* phi64 = nullptr;
    double* partials = nullptr;
    double* result = nullptr;
    unsigned* bad = nullptr;
    // graphs, one per starting buffer
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    int num_cus = 0;
};

namespace {

lbch_status ok() { return LBCH_OK; }

void drop_graphs(lbch_batch* b) {
    for (auto& e : b->exec) {
        if (e) (void)hipGraphExecDestroy(e);
        e = nullptr;
    }
}

void free_all(lbch_batch* b) {
    drop_graphs(b);
    for (void* p : {b->f[0], b->f[1], (void*)b->cfg[0].d_members, (void*)b->cfg[0].d_tile_member,
                    (void*)b->cfg[1].d_members, (void*)b->cfg[1].d_tile_member, (void*)b->d_counter,
                    (void*)b->phi64, (void*)b->partials, (void*)b->result, (void*)b->bad})
        if (p) (void)hipFree(p);
}

template <typename T>
BatchMember<T> make_desc(const Member& mm, const StepCoef<T>& c, int hc, int nt, int depth, int tile_begin) {
    BatchMember<T> d{};
    d.g = mm.g;
    d.base = mm.base;
    d.c = c;
    const int W = nt - 8 * depth;
    d.strips = (mm.g.nx + W - 1) / W;
    d.hc = std::min(hc, mm.g.ny);
    d.chunks = (mm.g.ny + d.hc - 1) / d.hc;
    d.tile_begin = tile_begin;
    return d;
}

// (Re)builds descriptors, the tile list (largest members first) and the persistent grid of one depth.
lbch_status configure(lbch_batch* b, int depth, int nt, int hc_user, int blocks_user) {
    const int n = (int)b->m.size();
    BatchConfig& cf = b->cfg[depth - 1];
    const int hc_default = depth == 2 ? 64 : 32;   // a two-step sweep restarts 14 rows per chunk
    int hc = hc_user > 0 ? hc_user : hc_default;
    if (hc_user <= 0 && b->num_cus > 0) {
        // small ensembles: fewer tiles than CUs at the default chunk, so a launch
        // lasts one chunk's sweep; take the shortest chunk (>= 4 rows) that keeps
        // at most 2.5 tiles per CU (the rule of the single-grid tiling)
        const int W = nt - 8 * depth;
        auto tiles_at = [&](int h) {
            long long t = 0;
            for (const Member& mm : b->m)
                t += (long long)((mm.g.nx + W - 1) / W) * ((mm.g.ny + h - 1) / h);
            return t;
        };
        if (tiles_at(hc_default) < b->num_cus)
            for (int h = 4; h <= hc_default; ++h)
                if (tiles_at(h) * 2 <= 5LL * b->num_cus) {
                    hc = h;
                    break;
                }
    }
    // order members by work, largest first, so the queue ends on small tiles
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
        return (long long)b->m[a].g.nx * b->m[a].g.ny > (long long)b->m[c].g.nx * b->m[c].g.ny;
    });
    std::vector<BatchMember<double>> dd(n);
    std::vector<BatchMember<float>> df(n);
    std::vector<int> tile_member;
    int tb = 0;
    for (int k : order) {
        const Member& mm = b->m[k];
        dd[k] = make_desc<double>(mm, mm.cd, hc, nt, depth, tb);
        df[k] = make_desc<float>(mm, mm.cf, hc, nt, depth, tb);
        const int nt_tiles = dd[k].strips * dd[k].chunks;
        tile_member.insert(tile_member.end(), nt_tiles, k);
        tb += nt_tiles;
    }
    cf.total_tiles = tb;
    drop_graphs(b);
    if (cf.d_members) (void)hipFree(cf.d_members);
    if (cf.d_tile_member) (void)hipFree(cf.d_tile_member);
    cf.d_members = nullptr;
    cf.d_tile_member = nullptr;
    const size_t desc_bytes = b->precision == LBCH_FP64 ? n * sizeof(BatchMember<double>) : n * sizeof(BatchMember<float>);
    HIP_TRY(hipMalloc(&cf.d_members, desc_bytes));
    HIP_TRY(hipMalloc((void**)&cf.d_tile_member, tile_member.size() * sizeof(int)));
    HIP_TRY(hipMemcpy(cf.d_members, b->precision == LBCH_FP64 ? (const void*)dd.data() : (const void*)df.data(),
                      desc_bytes, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(cf.d_tile_member, tile_member.data(), tile_member.size() * sizeof(int), hipMemcpyHostToDevice));
    b->unit_all = true;
    for (const Member& mm : b->m)
        if (!(b->precision == LBCH_FP64 ? mm.cd.unit : mm.cf.unit)) b->unit_all = false;
    int per_cu = batch_blocks_per_cu(b->precision, depth, nt, b->unit_all);
    int blocks = blocks_user > 0 ? blocks_user : per_cu * b->num_cus;
    cf.nblocks = std::max(1, std::min(blocks, cf.total_tiles));
    cf.nt = nt;
    cf.hc_user = hc_user;
    cf.hc = hc;
    cf.blocks_user = blocks_user;
    b->counter_dirty = true;
    return ok();
}

lbch_status check_member(const lbch_batch* b, int32_t member) {
    if (!b) return fail(LBCH_E_INVALID, "batch handle is NULL");
    if (member < 0 || member >= (int32_t)b->m.size())
        return fail(LBCH_E_INVALID, "member %d outside 0..%d", member, (int)b->m.size() - 1);
    return ok();
}

lbch_status check_ready(const lbch_batch* b) {
    if (!b) return fail(LBCH_E_INVALID, "batch handle is NULL");
    for (size_t k = 0; k < b->m.size(); ++k)
        if (!b->m[k].initialized) return fail(LBCH_E_STATE, "member %zu not initialised", k);
    return ok();
}

void* member_ptr(lbch_batch* b, int which, int member) {
    return (char*)b->f[which] + b->m[member].base * (long long)b->esize;
}

const void* coef_of(const lbch_batch* b, int member) {
    return b->precision == LBCH_FP64 ? (const void*)&b->m[member].cd : (const void*)&b->m[member].cf;
}

hipError_t launch_depth(lbch_batch* b, int depth, int from) {
    const BatchConfig& cf = b->cfg[depth - 1];
    return launch_batch_step(b->precision, depth, cf.nt, b->unit_all, b->f[from], b->f[from ^ 1], cf.d_members,
                             cf.d_tile_member, cf.total_tiles, cf.nblocks, b->d_counter + (depth - 1), b->stream);
}

lbch_status launch_one(lbch_batch* b, int depth, int from) {
    HIP_TRY(launch_depth(b, depth, from));
    return ok();
}

lbch_status reset_counter(lbch_batch* b) {
    if (b->counter_dirty) {
        HIP_TRY(launch_zero_u64(b->d_counter, 2, b->stream));
        b->counter_dirty = false;
    }
    return ok();
}

}  // namespace

extern "C" lbch_status lbch_batch_create(const lbch_params* members, int32_t count, void* hip_stream,
                                         lbch_batch** out) {
    if (!out) return fail(LBCH_E_INVALID, "out pointer is NULL");
    if (!members || count < 1) return fail(LBCH_E_INVALID, "need count >= 1 members");
    for (int k = 0; k < count; ++k) {
        lbch_status st = lbch_params_validate(&members[k]);
        if (st != LBCH_OK) return st;
        if (members[k].lattice != LBCH_D2Q9)
            return fail(LBCH_E_UNSUPPORTED, "member %d: ensembles hold D2Q9 grids only", k);
        if (members[k].precision != members[0].precision)
            return fail(LBCH_E_INVALID, "member %d precision differs from member 0", k);
    }
    lbch_batch* b = new (std::nothrow) lbch_batch();
    if (!b) return fail(LBCH_E_OOM, "host allocation failed");
    b->precision = members[0].precision;
    b->esize = b->precision == LBCH_FP64 ? 8 : 4;
    b->stream = (hipStream_t)hip_stream;
    b->m.resize(count);
    long long off = 0, max_nodes = 1;
    for (int k = 0; k < count; ++k) {
        Member& mm = b->m[k];
        mm.p = members[k];
        mm.g.nx = mm.p.nx;
        mm.g.ny = mm.p.ny;
        mm.g.pitch = (mm.p.nx + 63) / 64 * 64;
        mm.g.pad_ = 0;
        mm.g.plane = (long long)mm.g.pitch * mm.p.ny + 64;
        mm.base = off;
        off += (mm.g.plane * 9 + 63) / 64 * 64;
        fill_coef<double>(&mm.p, mm.cd);
        fill_coef<float>(&mm.p, mm.cf);
        fill_red(&mm.p, mm.rc);
        mm.initialized = false;
        max_nodes = std::max(max_nodes, (long long)mm.p.nx * mm.p.ny);
    }
    b->total_elems = off;
    {
        // as for one simulation: ensembles of at most 512^2 nodes in all run one
        // step per launch by default (latency-bound launches)
        long long nodes = 0;
        for (const Member& mm : b->m) nodes += (long long)mm.p.nx * mm.p.ny;
        b->depth = nodes <= 512LL * 512 ? 1 : 2;
    }
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&b->num_cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipMalloc(&b->f[0], off * b->esize);
    if (e == hipSuccess) e = hipMalloc(&b->f[1], off * b->esize);
    if (e == hipSuccess) e = hipMalloc((void**)&b->phi64, max_nodes * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void**)&b->partials, (size_t)kRedBlocks * 4 * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void**)&b->result, 8 * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void**)&b->bad, count * sizeof(unsigned));
    if (e == hipSuccess) e = hipMalloc((void**)&b->d_counter, 2 * sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMemset(b->bad, 0, count * sizeof(unsigned));
    if (e != hipSuccess) {
        free_all(b);
        delete b;
        (void)hipGetLastError();
        return fail(e == hipErrorOutOfMemory ? LBCH_E_OOM : LBCH_E_DEVICE, "batch allocation failed: %s",
                    hipGetErrorString(e));
    }
    lbch_status st = configure(b, 1, 128, 0, 0);
    if (st == LBCH_OK) st = configure(b, 2, 128, 0, 0);
    if (st != LBCH_OK) {
        free_all(b);
        delete b;
        return st;
    }
    *out = b;
    return ok();
}

extern "C" lbch_status lbch_batch_destroy(lbch_batch* b) {
    if (!b) return ok();
    (void)hipStreamSynchronize(b->stream);
    free_all(b);
    delete b;
    return ok();
}

extern "C" lbch_status lbch_batch_init_device(lbch_batch* b, int32_t member, const void* phi0_dev, int32_t dtype,
                                              int64_t n) {
    lbch_status st = check_member(b, member);
    if (st != LBCH_OK) return st;
    if (!phi0_dev) return fail(LBCH_E_INVALID, "phi0 pointer is NULL");
    if (dtype != LBCH_FP64 && dtype != LBCH_FP32) return fail(LBCH_E_INVALID, "unknown dtype %d", dtype);
    Member& mm = b->m[member];
    if (n != (int64_t)mm.g.nx * mm.g.ny) return fail(LBCH_E_INVALID, "n = %lld does not match member grid", (long long)n);
    HIP_TRY(launch_zero_u32(b->bad + member, 1, b->stream));
    HIP_TRY(launch_init(b->precision, phi0_dev, dtype, member_ptr(b, b->cur, member), mm.g, coef_of(b, member),
                        b->bad + member, b->stream));
    mm.initialized = true;
    return ok();
}

extern "C" lbch_status lbch_batch_init(lbch_batch* b, int32_t member, const double* phi0, int64_t n) {
    lbch_status st = check_member(b, member);
    if (st != LBCH_OK) return st;
    if (!phi0) return fail(LBCH_E_INVALID, "phi0 pointer is NULL");
    Member& mm = b->m[member];
    const int64_t nn = (int64_t)mm.g.nx * mm.g.ny;
    if (n != nn) return fail(LBCH_E_INVALID, "n = %lld but member %d has %lld nodes", (long long)n, member, (long long)nn);
    for (int64_t i = 0; i < nn; ++i)
        if (!std::isfinite(phi0[i])) return fail(LBCH_E_INVALID, "phi0[%lld] is not finite", (long long)i);
    HIP_TRY(hipMemcpyAsync(b->phi64, phi0, nn * sizeof(double), hipMemcpyHostToDevice, b->stream));
    st = lbch_batch_init_device(b, member, b->phi64, LBCH_FP64, n);
    if (st != LBCH_OK) return st;
    HIP_TRY(hipStreamSynchronize(b->stream));
    return ok();
}

extern "C" lbch_status lbch_batch_step(lbch_batch* b, int64_t nsteps) {
    lbch_status st = check_ready(b);
    if (st != LBCH_OK) return st;
    if (nsteps < 0) return fail(LBCH_E_INVALID, "nsteps = %lld < 0", (long long)nsteps);
    st = reset_counter(b);
    if (st != LBCH_OK) return st;
    const int depth = b->depth;
    const int64_t graph_steps = (int64_t)kGraphLaunches * depth;
    int64_t left = nsteps;
    if (b->stream != nullptr && left >= graph_steps) {
        if (!b->exec[b->cur]) {
            hipGraph_t graph = nullptr;
            HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
            int from = b->cur;
            for (int k = 0; k < kGraphLaunches; ++k) {
                hipError_t e = launch_depth(b, depth, from);
                if (e != hipSuccess) {
                    (void)hipStreamEndCapture(b->stream, &graph);
                    if (graph) (void)hipGraphDestroy(graph);
                    return fail(LBCH_E_DEVICE, "capture failed: %s", hipGetErrorString(e));
                }
                from ^= 1;
            }
            HIP_TRY(hipStreamEndCapture(b->stream, &graph));
            hipError_t e = hipGraphInstantiate(&b->exec[b->cur], graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) return fail(LBCH_E_DEVICE, "graph instantiate failed: %s", hipGetErrorString(e));
        }
        while (left >= graph_steps) {
            HIP_TRY(hipGraphLaunch(b->exec[b->cur], b->stream));
            left -= graph_steps;
            b->step += graph_steps;
        }
    }
    while (left > 0) {
        const int d = left >= depth ? depth : 1;
        st = launch_one(b, d, b->cur);
        if (st != LBCH_OK) return st;
        b->cur ^= 1;
        b->step += d;
        left -= d;
    }
    return ok();
}

extern "C" lbch_status lbch_batch_get_step(const lbch_batch* b, int64_t* step) {
    if (!b || !step) return fail(LBCH_E_INVALID, "NULL argument");
    *step = b->step;
    return ok();
}

extern "C" lbch_status lbch_batch_synchronize(lbch_batch* b) {
    if (!b) return fail(LBCH_E_INVALID, "batch handle is NULL");
    HIP_TRY(hipStreamSynchronize(b->stream));
    return ok();
}

namespace {

lbch_status member_phi(lbch_batch* b, int member, double out4[4]) {
    Member& mm = b->m[member];
    HIP_TRY(launch_moments(b->precision, member_ptr(b, b->cur, member), mm.g, b->phi64, 0, b->partials, kRedBlocks,
                           b->stream));
    const int kinds[4] = {0, 1, 2, 0};
    HIP_TRY(launch_finalize(b->partials, kRedBlocks, 4, kinds, b->result, b->stream));
    HIP_TRY(hipMemcpyAsync(out4, b->result, 4 * sizeof(double), hipMemcpyDeviceToHost, b->stream));
    unsigned bad = 0;
    HIP_TRY(hipMemcpyAsync(&bad, b->bad + member, sizeof bad, hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    if (bad) out4[3] += bad;
    return ok();
}

}  // namespace

extern "C" lbch_status lbch_batch_moments(lbch_batch* b, int32_t member, double* phi_out, double* mass,
                                          double* phi_min, double* phi_max) {
    lbch_status st = check_member(b, member);
    if (st != LBCH_OK) return st;
    if (!b->m[member].initialized) return fail(LBCH_E_STATE, "member %d not initialised", member);
    double r[4];
    st = member_phi(b, member, r);
    if (st != LBCH_OK) return st;
    const Member& mm = b->m[member];
    if (phi_out)
        HIP_TRY(hipMemcpy(phi_out, b->phi64, (size_t)mm.g.nx * mm.g.ny * sizeof(double), hipMemcpyDeviceToHost));
    if (mass) *mass = r[0] * mm.p.dx * mm.p.dx;
    if (phi_min) *phi_min = r[1];
    if (phi_max) *phi_max = r[2];
    if (r[3] != 0.0) return fail(LBCH_E_NONFINITE, "member %d holds %.0f non-finite phi values", member, r[3]);
    return ok();
}

extern "C" lbch_status lbch_batch_free_energy(lbch_batch* b, int32_t member, double* energy, double* terms4) {
    lbch_status st = check_member(b, member);
    if (st != LBCH_OK) return st;
    if (!b->m[member].initialized) return fail(LBCH_E_STATE, "member %d not initialised", member);
    double r[4];
    st = member_phi(b, member, r);
    if (st != LBCH_OK) return st;
    const Member& mm = b->m[member];
    HIP_TRY(launch_energy(b->phi64, mm.g, mm.rc, b->partials, kRedBlocks, b->stream));
    const int kinds[4] = {0, 0, 0, 0};
    HIP_TRY(launch_finalize(b->partials, kRedBlocks, 4, kinds, b->result, b->stream));
    double e[4];
    HIP_TRY(hipMemcpyAsync(e, b->result, 4 * sizeof(double), hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    const double a = mm.rc.area;
    if (energy) *energy = (e[0] + e[1] + e[2]) * a;
    if (terms4) {
        terms4[0] = e[0] * a;
        terms4[1] = e[1] * a;
        terms4[2] = e[2] * a;
        terms4[3] = (e[0] + e[1] + e[2]) * a;
    }
    if (r[3] != 0.0 || e[3] != 0.0) return fail(LBCH_E_NONFINITE, "free energy of a non-finite member %d", member);
    return ok();
}

extern "C" lbch_status lbch_batch_phi_device(lbch_batch* b, int32_t member, void* dst, int32_t dtype) {
    lbch_status st = check_member(b, member);
    if (st != LBCH_OK) return st;
    if (!b->m[member].initialized) return fail(LBCH_E_STATE, "member %d not initialised", member);
    if (!dst) return fail(LBCH_E_INVALID, "dst is NULL");
    if (dtype != LBCH_FP64 && dtype != LBCH_FP32) return fail(LBCH_E_INVALID, "unknown dtype %d", dtype);
    HIP_TRY(launch_moments(b->precision, member_ptr(b, b->cur, member), b->m[member].g, dst, dtype, b->partials,
                           kRedBlocks, b->stream));
    return ok();
}

extern "C" lbch_status lbch_batch_set_time_blocking(lbch_batch* b, int32_t depth) {
    if (!b) return fail(LBCH_E_INVALID, "batch handle is NULL");
    if (depth != 1 && depth != 2) return fail(LBCH_E_INVALID, "time-blocking depth %d not in {1, 2}", depth);
    if (depth != b->depth) drop_graphs(b);
    b->depth = depth;
    return ok();
}

extern "C" lbch_status lbch_batch_get_time_blocking(const lbch_batch* b, int32_t* depth) {
    if (!b || !depth) return fail(LBCH_E_INVALID, "NULL argument");
    *depth = b->depth;
    return ok();
}

extern "C" lbch_status lbch_batch_set_tiling(lbch_batch* b, int32_t block_threads, int32_t rows_per_block,
                                             int32_t persistent_blocks) {
    if (!b) return fail(LBCH_E_INVALID, "batch handle is NULL");
    if (block_threads != 0 && block_threads != 64 && block_threads != 128 && block_threads != 256 &&
        block_threads != 512)
        return fail(LBCH_E_INVALID, "block_threads %d not in {64, 128, 256, 512}", block_threads);
    if (b->depth == 2 && (block_threads == 64 || (b->precision == LBCH_FP64 && block_threads == 512)))
        return fail(LBCH_E_INVALID, "block_threads %d not available at time-blocking depth 2", block_threads);
    if (rows_per_block < 0 || persistent_blocks < 0) return fail(LBCH_E_INVALID, "negative tiling argument");
    HIP_TRY(hipStreamSynchronize(b->stream));
    return configure(b, b->depth, block_threads ? block_threads : 128, rows_per_block, persistent_blocks);
}

extern "C" lbch_status lbch_batch_get_tiling(const lbch_batch* b, int32_t* block_threads, int32_t* rows_per_block,
                                             int32_t* persistent_blocks, int32_t* total_tiles) {
    if (!b) return fail(LBCH_E_INVALID, "batch handle is NULL");
    const BatchConfig& cf = b->cfg[b->depth - 1];
    if (block_threads) *block_threads = cf.nt;
    if (rows_per_block) *rows_per_block = cf.hc;
    if (persistent_blocks) *persistent_blocks = cf.nblocks;
    if (total_tiles) *total_tiles = cf.total_tiles;
    return ok();
}

extern "C" lbch_status lbch_batch_nodes(const lbch_batch* b, int64_t* nodes) {
    if (!b || !nodes) return fail(LBCH_E_INVALID, "NULL argument");
    int64_t s = 0;
    for (const Member& mm : b->m) s += (int64_t)mm.g.nx * mm.g.ny;
    *nodes = s;
    return ok();
}

extern "C" lbch_status lbch_batch_autotune(lbch_batch* b, int32_t steps_per_trial, int32_t* block_threads,
                                           int32_t* rows_per_block, double* ms_per_step) {
    lbch_status st = check_ready(b);
    if (st != LBCH_OK) return st;
    if (steps_per_trial < 1) return fail(LBCH_E_INVALID, "steps_per_trial %d < 1", steps_per_trial);
    HIP_TRY(hipStreamSynchronize(b->stream));
    hipEvent_t a = nullptr, e2 = nullptr;
    HIP_TRY(hipEventCreate(&a));
    HIP_TRY(hipEventCreate(&e2));
    float best[2] = {-1.0f, -1.0f};                 // per step, per depth
    int best_nt[2] = {b->cfg[0].nt, b->cfg[1].nt}, best_hc[2] = {b->cfg[0].hc_user, b->cfg[1].hc_user};
    for (int depth = 1; depth <= 2 && st == LBCH_OK; ++depth) {
        for (int nt : {64, 128, 256}) {
            if (depth == 2 && nt == 64) continue;
            for (int hc : {0, 16, 32, 64, 128}) {        // 0: the default rule's height
                if (depth == 2 && hc > 0 && hc < 32) continue;
                st = configure(b, depth, nt, hc, b->cfg[depth - 1].blocks_user);
                if (st == LBCH_OK) st = reset_counter(b);
                if (st != LBCH_OK) break;
                // trials: state in f[cur] -> idle buffer, never swapped
                st = launch_one(b, depth, b->cur);
                hipError_t e = st == LBCH_OK ? hipEventRecord(a, b->stream) : hipErrorUnknown;
                for (int k = 0; e == hipSuccess && k < steps_per_trial; ++k) e = launch_depth(b, depth, b->cur);
                if (e == hipSuccess) e = hipEventRecord(e2, b->stream);
                if (e == hipSuccess) e = hipEventSynchronize(e2);
                float ms = 0.0f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, e2);
                if (e != hipSuccess) {
                    st = fail(LBCH_E_DEVICE, "batch autotune trial failed: %s", hipGetErrorString(e));
                    break;
                }
                ms /= (float)depth;
                if (best[depth - 1] < 0.0f || ms < best[depth - 1]) {
                    best[depth - 1] = ms;
                    best_nt[depth - 1] = nt;
                    best_hc[depth - 1] = hc;
                }
            }
            if (st != LBCH_OK) break;
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(e2);
    if (st != LBCH_OK) return st;
    for (int depth = 1; depth <= 2; ++depth) {
        st = configure(b, depth, best_nt[depth - 1], best_hc[depth - 1], b->cfg[depth - 1].blocks_user);
        if (st != LBCH_OK) return st;
    }
    const int d = (best[1] >= 0.0f && best[1] < best[0]) ? 2 : 1;
    if (d != b->depth) drop_graphs(b);
    b->depth = d;
    if (block_threads) *block_threads = best_nt[d - 1];
    if (rows_per_block) *rows_per_block = b->cfg[d - 1].hc;   // the height in use
    if (ms_per_step) *ms_per_step = best[d - 1] / steps_per_trial;
    return ok();
}

lbch_status lbch_batch_load_window(lbch_batch* b, int member, const lbch_sim* s, int y0, int x0) {
    lbch_status st = check_member(b, member);
    if (st != LBCH_OK) return st;
    if (!s || !s->initialized) return fail(LBCH_E_STATE, "source simulation not initialised");
    if (s->d3) return fail(LBCH_E_UNSUPPORTED, "windows are taken from D2Q9 simulations only");
    if (s->precision != b->precision) return fail(LBCH_E_INVALID, "precision mismatch");
    HIP_TRY(launch_copy_window(b->precision, s->f[s->cur], s->g, y0, x0, member_ptr(b, b->cur, member),
                               b->m[member].g, b->stream));
    b->m[member].initialized = true;
    return ok();
}
