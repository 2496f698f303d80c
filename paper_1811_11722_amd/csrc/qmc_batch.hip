// Batched estimates: many plans (sectors of different d, n, m) in one
// persistent, graph-replayed launch.
//
// The batch context concatenates every plan's generating vector, stride
// steps, shifts and parameter blob into device arrays once, cuts the work
// into tiles of tile_points lattice points times one shift tile, orders the
// tiles longest first (a cost model per plan: points times an evaluation
// cost from d and the polynomial sizes) and captures {counter reset,
// persistent kernel, per-plan finalize} into a HIP graph that later calls with
// the same plans and parameters replay.  The comparison mode launches each
// plan's own lattice and finalize kernels instead, all on one stream with a
// single synchronisation at the end.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>

#include "qmc_runtime.hpp"

namespace qmc {

struct qmc_plan_extra {};

std::map<BatchKey, BatchLaunch> &batch_registry() {
    static std::map<BatchKey, BatchLaunch> reg;
    return reg;
}

namespace {

struct BatchCtx {
    std::vector<qmc_plan_s *> plans;
    std::vector<std::vector<double>> blobs;
    int key_family = 0;
    uint32_t np = 1, T = 4, tile_points = 0;
    uint32_t requested_tile_points = 0;  // the caller's option (0 = default): part of the context's key
    qmc_launch launch0{0, 0};            // the first plan's launch shape when built: part of the key
    int persistent = 0;  // 1: persistent workgroups, 0: one workgroup per tile
    int device = 0;
    hipStream_t stream = nullptr;
    struct Group {
        uint32_t d;
        BatchLaunch fn;
        uint32_t tile_begin, ntiles;
    };
    std::vector<Group> groups;  // one persistent launch per dimension
    // uniform batches (every plan with the same d, n and m): one launch of the
    // lattice kernel with the plans as instances along grid.y
    bool uniform = false;
    LatticeLaunch lfn = nullptr;
    LatticeArgs largs{};
    FinalizeArgs lfargs{};
    uint32_t lbx = 0, ltiles = 0;
    DeviceScratch dev;  // sectors, tiles, g, gstep, shifts, params, counter, partials, q, res
    BatchArgs args{};
    FinalizeBatchArgs fargs{};
    std::vector<BatchSector> hs;
    size_t nq = 0;
    double *h_q = nullptr, *h_res = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint32_t blocks = 0;
    ~BatchCtx() {
        if (stream) (void)hipStreamSynchronize(stream);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (h_q) (void)hipHostFree(h_q);
        if (h_res) (void)hipHostFree(h_res);
        if (stream) (void)hipStreamDestroy(stream);
    }
};

std::mutex g_batch_mu;
// qmc_batch_stats: table-driven contexts built, their graph launches,
// specialised graphs captured, their launches (under g_batch_mu)
uint64_t g_stats[4] = {0, 0, 0, 0};
std::vector<std::unique_ptr<BatchCtx>> g_batch;
constexpr size_t kMaxContexts = 8;

// evaluation cost of one point and shift, in arbitrary units
double plan_cost(int key_family, uint32_t d, const std::vector<double> &blob) {
    if (key_family == QMC_F_SECTOR || key_family == kFamSectorComplex) {
        uint64_t nu, nf;
        std::memcpy(&nu, &blob[0], 8);
        std::memcpy(&nf, &blob[1], 8);
        double factors = 0.0;
        for (uint64_t t = 0; t < nu + nf; ++t) {
            uint64_t c;
            const size_t at = t < nu ? kSectorHeader + nu + t : kSectorHeader + 2 * nu + (t - nu) + nf;
            std::memcpy(&c, &blob[at], 8);
            factors += (double)(c & 15u);
        }
        return 60.0 + 4.0 * d + 8.0 * (double)(nu + nf) + 8.0 * factors + (key_family == kFamSectorComplex ? 80 : 0);
    }
    return 20.0 + 12.0 * d;
}

qmc_status build_uniform(BatchCtx &c, uint32_t count, const qmc_plan_t *plans, const std::vector<Packed> &pk) {
    qmc_plan_s *p0 = plans[0];
    c.uniform = true;
    c.plans.assign(plans, plans + count);
    c.key_family = pk[0].key_family;
    c.np = pk[0].np;
    c.device = p0->device;
    for (uint32_t i = 0; i < count; ++i) c.blobs.push_back(pk[i].blob);
    // the first plan's launch configuration (qmc_plan_set_launch) applies to
    // the whole launch; otherwise shift tile 8 where 4 is the default
    uint32_t T = 0;
    const uint32_t want_T = p0->launch.shift_tile ? p0->launch.shift_tile
                                                  : (default_tile(c.key_family) == 4 ? 8 : default_tile(c.key_family));
    c.lfn = find_kernel(c.key_family, p0->tr, p0->d, want_T, T);
    if (!c.lfn)
        return fail(QMC_EUNSUPPORTED, "no kernel for family %d, transform %d/%d, d = %u", c.key_family, p0->tr.kind,
                    p0->tr.alpha, p0->d);
    const uint32_t d = p0->d, m = p0->m, n = p0->n, rows = padded_rows(m);
    c.T = T;
    c.ltiles = (m + T - 1) / T;
    if ((uint64_t)count * c.ltiles > 65535) return fail(QMC_EUNSUPPORTED, "too many instances for one launch");
    c.lbx = grid_x(n, count * c.ltiles, c.device, p0->launch.blocks_per_cu ? p0->launch.blocks_per_cu : 8);
    size_t pstride = 0;
    for (auto &b : pk) pstride = std::max(pstride, b.blob.size());
    std::vector<uint32_t> g((size_t)count * d), gs((size_t)count * d);
    std::vector<double> sh((size_t)count * rows * d), prm(count * pstride, 0.0);
    for (uint32_t i = 0; i < count; ++i) {
        std::copy(plans[i]->g.begin(), plans[i]->g.end(), g.begin() + (size_t)i * d);
        gstep_for(plans[i]->g.data(), d, n, (uint64_t)c.lbx * kBlock, &gs[(size_t)i * d]);
        const std::vector<double> ps = padded_shifts(plans[i]->shifts, m, d, rows, plans[i]->tr);
        std::copy(ps.begin(), ps.end(), sh.begin() + (size_t)i * rows * d);
        std::copy(pk[i].blob.begin(), pk[i].blob.end(), prm.begin() + (size_t)i * pstride);
        BatchSector s{};
        s.n = n;
        s.d = d;
        s.m = m;
        s.q_off = i * m * c.np;
        c.hs.push_back(s);
    }
    c.nq = (size_t)count * m * c.np;
    qmc_status st;
    if ((st = c.dev.alloc(g.size() * 4)) || (st = c.dev.alloc(gs.size() * 4)) || (st = c.dev.alloc(sh.size() * 8)) ||
        (st = c.dev.alloc(prm.size() * 8)) ||
        (st = c.dev.alloc((size_t)count * m * c.np * c.lbx * sizeof(double2))) || (st = c.dev.alloc(c.nq * 8)) ||
        (st = c.dev.alloc((size_t)count * 32)))
        return st;
    hipError_t e;
    if ((e = hipMemcpy(c.dev.ptr[0], g.data(), g.size() * 4, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(c.dev.ptr[1], gs.data(), gs.size() * 4, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(c.dev.ptr[2], sh.data(), sh.size() * 8, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(c.dev.ptr[3], prm.data(), prm.size() * 8, hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "batch upload");
    if ((e = hipHostMalloc((void **)&c.h_q, c.nq * 8, hipHostMallocDefault)) != hipSuccess ||
        (e = hipHostMalloc((void **)&c.h_res, (size_t)count * 32, hipHostMallocDefault)) != hipSuccess)
        return fail(QMC_ENOMEM, "hipHostMalloc: %s", hipGetErrorString(e));
    if ((e = hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking)) != hipSuccess)
        return hip_fail(e, "hipStreamCreate");
    LatticeArgs &a = c.largs;
    a.n = n;
    a.d = d;
    a.m = m;
    a.tiles = c.ltiles;
    a.inv_n = p0->inv_n;
    a.g = (const uint32_t *)c.dev.ptr[0];
    a.gstep = (const uint32_t *)c.dev.ptr[1];
    a.shifts = (const double *)c.dev.ptr[2];
    a.params = (const double *)c.dev.ptr[3];
    a.g_stride = d;
    a.shift_stride = rows * d;
    a.param_stride = (uint32_t)pstride;
    a.np = c.np;
    a.partials = (double2 *)c.dev.ptr[4];
    FinalizeArgs &f = c.lfargs;
    f.partials = a.partials;
    f.nblk = c.lbx;
    f.m = m;
    f.np = c.np;
    f.n = (double)n;
    f.scale = transform_scale(p0->tr, d);
    f.sub = 0.0;
    f.q = (double *)c.dev.ptr[5];
    f.res = (double *)c.dev.ptr[6];
    c.fargs.q = f.q;
    c.fargs.res = f.res;
    return QMC_OK;
}

qmc_status build_ctx(BatchCtx &c, uint32_t count, const qmc_plan_t *plans, const std::vector<Packed> &pk,
                     uint32_t tile_points) {
    qmc_plan_s *p0 = plans[0];
    c.plans.assign(plans, plans + count);
    c.key_family = pk[0].key_family;
    c.np = pk[0].np;
    c.device = p0->device;
    c.tile_points = tile_points;
    for (uint32_t i = 0; i < count; ++i) c.blobs.push_back(pk[i].blob);
    const int alpha = (p0->tr.kind == QMC_T_KOROBOV || p0->tr.kind == QMC_T_SIDI) ? p0->tr.alpha : 0;
    auto &reg = batch_registry();
    // one shift tile for the whole batch: the largest compiled for plan 0's d
    c.T = 0;
    for (int T : {4, 2, 1})
        if (reg.count(BatchKey{c.key_family, p0->tr.kind, alpha, (int)p0->d, T})) {
            c.T = (uint32_t)T;
            break;
        }
    std::map<uint32_t, BatchLaunch> fn_of_d;
    for (uint32_t i = 0; i < count && c.T; ++i) {
        auto it = reg.find(BatchKey{c.key_family, p0->tr.kind, alpha, (int)plans[i]->d, (int)c.T});
        if (it == reg.end())
            return fail(QMC_EUNSUPPORTED, "no batch kernel for family %d, transform %d/%d, d = %u", c.key_family,
                        p0->tr.kind, p0->tr.alpha, plans[i]->d);
        fn_of_d[plans[i]->d] = it->second;
    }
    if (!c.T)
        return fail(QMC_EUNSUPPORTED, "no batch kernel for family %d, transform %d/%d, d = %u", c.key_family,
                    p0->tr.kind, p0->tr.alpha, p0->d);
    const uint32_t T = c.T;

    std::vector<uint32_t> g, gs;
    std::vector<double> sh, prm;
    struct Work {
        double cost;
        uint32_t d;
        BatchTile t;
    };
    std::vector<Work> work;
    uint32_t slot = 0;
    size_t qoff = 0;
    for (uint32_t i = 0; i < count; ++i) {
        const qmc_plan_s *p = plans[i];
        BatchSector s{};
        s.n = p->n;
        s.d = p->d;
        s.m = p->m;
        s.jtiles = (p->n + tile_points - 1) / tile_points;
        s.inv_n = p->inv_n;
        s.scale = transform_scale(p->tr, p->d);
        s.g_off = (uint32_t)g.size();
        s.shift_off = (uint32_t)sh.size();
        s.param_off = (uint32_t)prm.size();
        s.slot_base = slot;
        s.q_off = (uint32_t)qoff;
        std::vector<uint32_t> step(p->d);
        gstep_for(p->g.data(), p->d, p->n, kBlock, step.data());
        g.insert(g.end(), p->g.begin(), p->g.end());
        gs.insert(gs.end(), step.begin(), step.end());
        const std::vector<double> psh = padded_shifts(p->shifts, p->m, p->d, (p->m + T - 1) / T * T, p->tr);
        sh.insert(sh.end(), psh.begin(), psh.end());
        prm.insert(prm.end(), pk[i].blob.begin(), pk[i].blob.end());
        const uint32_t ktiles = (p->m + T - 1) / T;
        const double cpp = plan_cost(c.key_family, p->d, pk[i].blob) * T;
        for (uint32_t kt = 0; kt < ktiles; ++kt)
            for (uint32_t jt = 0; jt < s.jtiles; ++jt) {
                const uint32_t pts = std::min(tile_points, p->n - jt * tile_points);
                work.push_back(Work{cpp * pts, p->d, BatchTile{i, kt * T, jt, 0}});
            }
        slot += ktiles * s.jtiles;
        qoff += (size_t)p->m * c.np;
        c.hs.push_back(s);
    }
    // group by dimension (groups with more work first), longest tiles first
    std::map<uint32_t, double> group_cost;
    for (const Work &w : work) group_cost[w.d] += w.cost;
    std::stable_sort(work.begin(), work.end(), [&](const Work &a, const Work &b) {
        if (a.d != b.d) return group_cost[a.d] != group_cost[b.d] ? group_cost[a.d] > group_cost[b.d] : a.d > b.d;
        return a.cost > b.cost;
    });
    std::vector<BatchTile> tiles(work.size());
    for (size_t t = 0; t < work.size(); ++t) {
        tiles[t] = work[t].t;
        if (c.groups.empty() || c.groups.back().d != work[t].d)
            c.groups.push_back(BatchCtx::Group{work[t].d, fn_of_d[work[t].d], (uint32_t)t, 0});
        c.groups.back().ntiles += 1;
    }
    c.nq = qoff;

    qmc_status st;
    const size_t psize = (size_t)slot * T * c.np * sizeof(double2);
    if ((st = c.dev.alloc(c.hs.size() * sizeof(BatchSector))) || (st = c.dev.alloc(tiles.size() * sizeof(BatchTile))) ||
        (st = c.dev.alloc(g.size() * 4)) || (st = c.dev.alloc(gs.size() * 4)) || (st = c.dev.alloc(sh.size() * 8)) ||
        (st = c.dev.alloc(prm.size() * 8)) || (st = c.dev.alloc(4 * c.groups.size() + 64)) ||
        (st = c.dev.alloc(psize)) ||
        (st = c.dev.alloc(qoff * 8)) || (st = c.dev.alloc((size_t)count * 32)))
        return st;
    hipError_t e;
    auto up = [&](int k, const void *src, size_t bytes) {
        return bytes ? hipMemcpy(c.dev.ptr[k], src, bytes, hipMemcpyHostToDevice) : hipSuccess;
    };
    if ((e = up(0, c.hs.data(), c.hs.size() * sizeof(BatchSector))) != hipSuccess ||
        (e = up(1, tiles.data(), tiles.size() * sizeof(BatchTile))) != hipSuccess ||
        (e = up(2, g.data(), g.size() * 4)) != hipSuccess || (e = up(3, gs.data(), gs.size() * 4)) != hipSuccess ||
        (e = up(4, sh.data(), sh.size() * 8)) != hipSuccess || (e = up(5, prm.data(), prm.size() * 8)) != hipSuccess)
        return hip_fail(e, "batch upload");
    if ((e = hipHostMalloc((void **)&c.h_q, std::max<size_t>(qoff, 1) * 8, hipHostMallocDefault)) != hipSuccess ||
        (e = hipHostMalloc((void **)&c.h_res, (size_t)count * 32, hipHostMallocDefault)) != hipSuccess)
        return fail(QMC_ENOMEM, "hipHostMalloc: %s", hipGetErrorString(e));
    if ((e = hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking)) != hipSuccess)
        return hip_fail(e, "hipStreamCreate");
    c.args.sectors = (const BatchSector *)c.dev.ptr[0];
    c.args.tiles = (const BatchTile *)c.dev.ptr[1];
    c.args.ntiles = (uint32_t)tiles.size();
    c.args.tile_points = tile_points;
    c.args.g = (const uint32_t *)c.dev.ptr[2];
    c.args.gstep = (const uint32_t *)c.dev.ptr[3];
    c.args.shifts = (const double *)c.dev.ptr[4];
    c.args.params = (const double *)c.dev.ptr[5];
    c.args.counter = (uint32_t *)c.dev.ptr[6];
    c.args.partials = (double2 *)c.dev.ptr[7];
    c.fargs.sectors = c.args.sectors;
    c.fargs.partials = c.args.partials;
    c.fargs.T = T;
    c.fargs.np = c.np;
    c.fargs.q = (double *)c.dev.ptr[8];
    c.fargs.res = (double *)c.dev.ptr[9];
    c.blocks = (uint32_t)device_cu_count(c.device) * 8;
    return QMC_OK;
}

hipError_t enqueue_batch(BatchCtx &c) {
    if (c.uniform) {
        hipError_t e = c.lfn(c.largs, dim3(c.lbx, (uint32_t)c.plans.size() * c.ltiles), c.stream);
        if (e == hipSuccess) e = launch_finalize(c.lfargs, (uint32_t)c.plans.size(), c.stream);
        return e;
    }
    hipError_t e = launch_zero_u32(c.args.counter, (uint32_t)c.groups.size(), c.stream);
    for (size_t gi = 0; gi < c.groups.size() && e == hipSuccess; ++gi) {
        BatchArgs a = c.args;
        a.tiles = c.args.tiles + c.groups[gi].tile_begin;
        a.ntiles = c.groups[gi].ntiles;
        a.counter = c.args.counter + gi;
        const uint32_t blocks = std::min<uint32_t>(c.blocks, a.ntiles);
        e = c.groups[gi].fn(a, blocks, c.persistent, c.stream);
    }
    if (e == hipSuccess) e = launch_finalize_batch(c.fargs, (uint32_t)c.plans.size(), c.stream);
    return e;
}

qmc_status run_graph(BatchCtx &c, bool use_graph) {
    hipError_t e;
    if (!use_graph) {
        e = enqueue_batch(c);
        return e == hipSuccess ? QMC_OK : hip_fail(e, "batch launch");
    }
    if (!c.exec) {
        e = hipStreamBeginCapture(c.stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "begin capture");
        hipError_t le = enqueue_batch(c);
        e = hipStreamEndCapture(c.stream, &c.graph);
        if (le != hipSuccess) return hip_fail(le, "capture launches");
        if (e != hipSuccess) return hip_fail(e, "end capture");
        e = hipGraphInstantiate(&c.exec, c.graph, nullptr, nullptr, 0);
        if (e != hipSuccess) return hip_fail(e, "graph instantiate");
    }
    e = hipGraphLaunch(c.exec, c.stream);
    if (e == hipSuccess) ++g_stats[1];
    return e == hipSuccess ? QMC_OK : hip_fail(e, "graph launch");
}

// A context is reused for the same plans, parameter blobs, requested tile
// size (which also decides between the uniform and the tiled layout),
// schedule and first plan's launch shape (the uniform launch takes it).
bool same_ctx(const BatchCtx &c, uint32_t count, const qmc_plan_t *plans, const std::vector<Packed> &pk,
              uint32_t requested_tile_points, int persistent) {
    if (c.plans.size() != count || c.requested_tile_points != requested_tile_points ||
        c.key_family != pk[0].key_family || c.persistent != persistent ||
        c.launch0.shift_tile != plans[0]->launch.shift_tile || c.launch0.blocks_per_cu != plans[0]->launch.blocks_per_cu)
        return false;
    for (uint32_t i = 0; i < count; ++i)
        if (c.plans[i] != plans[i] || c.blobs[i] != pk[i].blob) return false;
    return true;
}

}  // namespace

void plan_release_extra(qmc_plan_s *p) {
    std::lock_guard<std::mutex> lock(g_batch_mu);
    g_batch.erase(std::remove_if(g_batch.begin(), g_batch.end(),
                                 [p](const std::unique_ptr<BatchCtx> &c) {
                                     return std::find(c->plans.begin(), c->plans.end(), p) != c->plans.end();
                                 }),
                  g_batch.end());
    delete p->extra;
    p->extra = nullptr;
}

// One launch per plan of its run-time specialised sector kernel (each plan's
// own stream and buffers), then one synchronisation per plan's stream.
// Launch shape of one plan's specialised sector kernel, as plan_enqueue
// chooses it (the plan's own configuration, else T = 4 for real sectors of
// d <= 8, 1 with a deformation, 2 otherwise, and 16 workgroups per CU).
struct SpecPlan {
    hipFunction_t fn = nullptr;
    uint32_t T = 0, bx = 0, tiles = 0;
};

static qmc_status spec_prepare(qmc_plan_s *p, const Packed &pk, SpecPlan &sp) {
    const bool wide = !pk.cplx && p->d <= (pk.orders < 2 ? 8u : 6u);
    sp.T = p->launch.shift_tile ? p->launch.shift_tile : (pk.deform ? 1u : wide ? 4u : 2u);
    std::string err;
    sp.fn = jit_kernel(pk.blob, p->d, p->tr, sp.T, pk.cplx, p->device, err);
    if (!sp.fn) return fail(QMC_EUNSUPPORTED, "specialised sector kernel: %s", err.c_str());
    if (p->m * pk.np > kMaxRows) return fail(QMC_EUNSUPPORTED, "m * parts > %u", kMaxRows);
    sp.tiles = (p->m + sp.T - 1) / sp.T;
    sp.bx = grid_x(p->n, sp.tiles, p->device, p->launch.blocks_per_cu ? p->launch.blocks_per_cu : 16);
    qmc_status st = plan_upload_params(p, pk);
    if (!st) st = plan_set_gstep(p, sp.bx * kBlock);
    if (!st)
        st = ensure_buffer((void **)&p->d_partials, p->partials_cap, (size_t)p->m * pk.np * sp.bx * sizeof(double2),
                           "partials");
    return st;
}

// lattice kernel, finalize kernel and the copy of the results to the
// plan's pinned mirror, on stream s
static hipError_t spec_enqueue(qmc_plan_s *p, const Packed &pk, const SpecPlan &sp, hipStream_t s) {
    LatticeArgs a{};
    a.n = p->n;
    a.d = p->d;
    a.m = p->m;
    a.tiles = sp.tiles;
    a.inv_n = p->inv_n;
    a.g = p->d_g;
    a.gstep = p->d_gstep;
    a.shifts = p->d_shifts;
    a.params = p->d_params;
    a.g_stride = a.shift_stride = a.param_stride = 0;
    a.np = pk.np;
    a.partials = p->d_partials;
    hipError_t e = jit_launch(sp.fn, a, dim3(sp.bx, sp.tiles), s);
    if (e != hipSuccess) return e;
    FinalizeArgs f{};
    f.partials = p->d_partials;
    f.nblk = sp.bx;
    f.m = p->m;
    f.np = pk.np;
    f.n = (double)p->n;
    f.scale = transform_scale(p->tr, p->d);
    f.sub = 0.0;
    f.q = p->d_out;
    f.res = p->d_out + out_res_offset(p->m);
    if ((e = launch_finalize(f, 1, s)) != hipSuccess) return e;
    return hipMemcpyAsync(p->h_out, p->d_out, out_doubles(p->m) * sizeof(double), hipMemcpyDeviceToHost, s);
}

// A captured specialised schedule: the kernels of every plan on kSpecChains
// parallel chains of one graph, valid while the plans keep the buffers,
// kernels and launch shapes it was captured with.
constexpr int kSpecChains = 4;
struct SpecCtx {
    std::vector<qmc_plan_s *> plans;
    std::vector<SpecPlan> sp;
    std::vector<std::vector<const void *>> bufs;  // per plan: params, partials, out, gstep, g, shifts, h_out
    hipStream_t stream = nullptr;
    hipStream_t side[kSpecChains] = {};
    hipEvent_t fork = nullptr, join[kSpecChains] = {};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~SpecCtx() {
        if (stream) (void)hipStreamSynchronize(stream);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (fork) (void)hipEventDestroy(fork);
        for (int c = 0; c < kSpecChains; ++c) {
            if (join[c]) (void)hipEventDestroy(join[c]);
            if (side[c]) (void)hipStreamDestroy(side[c]);
        }
        if (stream) (void)hipStreamDestroy(stream);
    }
};
std::vector<std::unique_ptr<SpecCtx>> g_spec;

static std::vector<const void *> spec_buffers(qmc_plan_s *p) {
    return {p->d_params, p->d_partials, p->d_out, p->d_gstep, p->d_g, p->d_shifts, p->h_out};
}

static qmc_status spec_capture(SpecCtx &c, const std::vector<Packed> &pk) {
    hipError_t e = hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c.fork, hipEventDisableTiming);
    for (int k = 0; k < kSpecChains && e == hipSuccess; ++k) {
        e = hipStreamCreateWithFlags(&c.side[k], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c.join[k], hipEventDisableTiming);
    }
    if (e != hipSuccess) return hip_fail(e, "specialised batch streams");
    if ((e = hipStreamBeginCapture(c.stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
        return hip_fail(e, "begin capture");
    hipError_t ce = hipEventRecord(c.fork, c.stream);
    for (int k = 0; k < kSpecChains && ce == hipSuccess; ++k) ce = hipStreamWaitEvent(c.side[k], c.fork, 0);
    for (size_t i = 0; i < c.plans.size() && ce == hipSuccess; ++i)
        ce = spec_enqueue(c.plans[i], pk[i], c.sp[i], c.side[i % kSpecChains]);
    for (int k = 0; k < kSpecChains && ce == hipSuccess; ++k) {
        ce = hipEventRecord(c.join[k], c.side[k]);
        if (ce == hipSuccess) ce = hipStreamWaitEvent(c.stream, c.join[k], 0);
    }
    e = hipStreamEndCapture(c.stream, &c.graph);
    if (ce != hipSuccess) return hip_fail(ce, "capture specialised batch");
    if (e != hipSuccess) return hip_fail(e, "end capture");
    if ((e = hipGraphInstantiate(&c.exec, c.graph, nullptr, nullptr, 0)) != hipSuccess)
        return hip_fail(e, "instantiate graph");
    return QMC_OK;
}

// One launch per plan of its run-time specialised kernel (sectors only):
// without a graph on the plans' own streams, with one a captured graph that
// later calls with the same plans, structures and buffers replay (the
// parameter blobs are uploaded before every replay, so new coefficients
// with the same exponent structure reuse it).
static qmc_status batch_specialised(uint32_t count, const qmc_plan_t *plans, const std::vector<Packed> &pk,
                                    qmc_result *out, bool use_graph) {
    qmc_status first_bad = QMC_OK;
    if (!use_graph) {
        for (uint32_t i = 0; i < count; ++i) {
            qmc_plan_s *p = plans[i];
            const int32_t jit = p->jit_mode;
            p->jit_mode = 2;  // specialised kernel or an error
            qmc_status st = plan_enqueue(p, pk[i], p->launch.shift_tile, p->launch.blocks_per_cu);
            p->jit_mode = jit;
            if (st) return st;
        }
        for (uint32_t i = 0; i < count; ++i) {
            qmc_status st = plan_collect(plans[i], pk[i].np, &out[i], nullptr, pk[i].crossing);
            if (st == QMC_ENONFINITE || st == QMC_ECONTOUR) {
                if (!first_bad || st == QMC_ENONFINITE) first_bad = st;
            } else if (st) {
                return st;
            }
        }
        return first_bad;
    }
    std::vector<SpecPlan> sp(count);
    for (uint32_t i = 0; i < count; ++i) {
        qmc_status st = spec_prepare(plans[i], pk[i], sp[i]);
        if (st) return st;
    }
    std::lock_guard<std::mutex> lock(g_batch_mu);
    SpecCtx *c = nullptr;
    for (auto &x : g_spec) {
        if (x->plans.size() != count || !std::equal(x->plans.begin(), x->plans.end(), plans)) continue;
        bool same = true;
        for (uint32_t i = 0; i < count && same; ++i)
            same = x->sp[i].fn == sp[i].fn && x->sp[i].T == sp[i].T && x->sp[i].bx == sp[i].bx &&
                   x->bufs[i] == spec_buffers(plans[i]);
        if (same) c = x.get();
    }
    if (!c) {
        auto fresh = std::make_unique<SpecCtx>();
        fresh->plans.assign(plans, plans + count);
        fresh->sp = sp;
        for (uint32_t i = 0; i < count; ++i) fresh->bufs.push_back(spec_buffers(plans[i]));
        qmc_status st = spec_capture(*fresh, pk);
        if (st) return st;
        ++g_stats[2];
        if (g_spec.size() >= kMaxContexts) g_spec.erase(g_spec.begin());
        g_spec.push_back(std::move(fresh));
        c = g_spec.back().get();
    }
    // the blobs went up on each plan's own stream in spec_prepare, which
    // waited for them
    hipError_t e = hipGraphLaunch(c->exec, c->stream);
    if (e == hipSuccess) ++g_stats[3];
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "specialised batch graph");
    for (uint32_t i = 0; i < count; ++i) {
        qmc_plan_s *p = plans[i];
        p->last_T = sp[i].T;
        p->last_bx = sp[i].bx;
        p->last_jit = true;
        qmc_status st = plan_results(p, pk[i].np, &out[i], nullptr, pk[i].crossing);
        if (st == QMC_ENONFINITE || st == QMC_ECONTOUR) {
            if (!first_bad || st == QMC_ENONFINITE) first_bad = st;
        } else if (st) {
            return st;
        }
    }
    return first_bad;
}

}  // namespace qmc

using namespace qmc;

extern "C" {

qmc_status qmc_integrate_batch(uint32_t count, const qmc_plan_t *plans, qmc_family family, const void *const *params,
                               const qmc_batch_opts *opts, qmc_result *out) {
    if (count == 0) return fail(QMC_EINVAL, "count must be >= 1");
    if (!plans || !params || !out) return fail(QMC_EINVAL, "null argument");
    const qmc_batch_opts o = opts ? *opts : qmc_batch_opts{1, 0, 0, QMC_BATCH_DEFAULT};
    uint32_t tile_points = o.tile_points ? o.tile_points : 8192;
    if (tile_points % kBlock) return fail(QMC_EINVAL, "tile_points must be a multiple of %d", kBlock);
    if (o.schedule < QMC_BATCH_DEFAULT || o.schedule > QMC_BATCH_SPECIALISED)
        return fail(QMC_EINVAL, "unknown schedule %d", o.schedule);
    const bool specialised = o.schedule == QMC_BATCH_SPECIALISED;
    if (specialised && family != QMC_F_SECTOR)
        return fail(QMC_EUNSUPPORTED, "the specialised schedule is built for QMC_F_SECTOR");
    const int persistent = o.schedule == QMC_BATCH_PERSISTENT;
    std::vector<Packed> pk(count);
    for (uint32_t i = 0; i < count; ++i) {
        if (!plans[i]) return fail(QMC_EINVAL, "plan %u is NULL", i);
        if (plans[i]->tr.kind != plans[0]->tr.kind || plans[i]->tr.alpha != plans[0]->tr.alpha)
            return fail(QMC_EINVAL, "plan %u has a different transform", i);
        if (plans[i]->device != plans[0]->device) return fail(QMC_EINVAL, "plans on different devices");
        qmc_status st = pack_params((int)family, plans[i]->d, params[i], pk[i]);
        if (st) return st;
        if (pk[i].key_family != pk[0].key_family) return fail(QMC_EINVAL, "mixed real and complex sectors");
        if (pk[i].orders >= 2) return fail(QMC_EUNSUPPORTED, "batches take the plain integrand (n_orders < 2)");
        if (pk[i].deform && !specialised)
            return fail(QMC_EUNSUPPORTED, "deformed sectors need the specialised schedule");
        if (plans[i]->m * pk[i].np > kMaxRows) return fail(QMC_EUNSUPPORTED, "m * parts > %u", kMaxRows);
    }

    if (specialised) return batch_specialised(count, plans, pk, out, o.use_graph != 0);

    std::lock_guard<std::mutex> lock(g_batch_mu);
    BatchCtx *c = nullptr;
    for (auto &x : g_batch)
        if (same_ctx(*x, count, plans, pk, o.tile_points, persistent)) c = x.get();
    if (!c) {
        auto fresh = std::make_unique<BatchCtx>();
        bool uniform = o.tile_points == 0 && count * ((plans[0]->m + 7) / 8) <= 65535;
        for (uint32_t i = 1; i < count && uniform; ++i)
            uniform = plans[i]->d == plans[0]->d && plans[i]->n == plans[0]->n && plans[i]->m == plans[0]->m;
        qmc_status st = uniform ? build_uniform(*fresh, count, plans, pk)
                                : build_ctx(*fresh, count, plans, pk, tile_points);
        if (st) return st;
        fresh->persistent = persistent;
        fresh->requested_tile_points = o.tile_points;
        fresh->launch0 = plans[0]->launch;
        ++g_stats[0];
        if (g_batch.size() >= kMaxContexts) g_batch.erase(g_batch.begin());
        g_batch.push_back(std::move(fresh));
        c = g_batch.back().get();
    }

    hipError_t e;
    bool any_nonfinite = false;
    if (o.per_plan_launches) {
        // comparison mode: each plan's own table-driven kernels, one stream
        for (uint32_t i = 0; i < count; ++i) {
            qmc_plan_s *p = plans[i];
            hipStream_t keep = p->stream;
            const int32_t jit = p->jit_mode;
            p->stream = c->stream;
            p->jit_mode = 0;
            qmc_status st = plan_enqueue(p, pk[i], c->T, 0);
            if (!st && (e = hipMemcpyAsync(p->h_out, p->d_out, out_doubles(p->m) * sizeof(double),
                                           hipMemcpyDeviceToHost, c->stream)) != hipSuccess)
                st = hip_fail(e, "copy results");
            p->stream = keep;
            p->jit_mode = jit;
            if (st) return st;
        }
        if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return hip_fail(e, "synchronize");
        for (uint32_t i = 0; i < count; ++i) {
            qmc_plan_s *p = plans[i];
            const double *q = p->h_out, *res = p->h_out + out_res_offset(p->m);
            bool fin = true;
            for (uint32_t k = 0; k < p->m * pk[i].np; ++k) fin = fin && std::isfinite(q[k]);
            out[i] = qmc_result{res[0], pk[i].np == 2 ? res[1] : 0.0, res[2], pk[i].np == 2 ? res[3] : 0.0,
                                (int32_t)(pk[i].np == 2), 0, 0.0};
            if (!fin) {
                out[i].mean_re = out[i].mean_im = out[i].err_re = out[i].err_im = NAN;
                any_nonfinite = true;
            }
        }
    } else {
        // with timing on the first plan, the device time of the batch's
        // kernels (graph launch to its end, on the batch stream) is added to
        // that plan's kernel time
        qmc_plan_s *p0 = plans[0];
        if (p0->timing) (void)hipEventRecord(p0->ev0, c->stream);
        qmc_status st = run_graph(*c, o.use_graph != 0);
        if (st) return st;
        if (p0->timing) (void)hipEventRecord(p0->ev1, c->stream);
        if ((e = hipMemcpyAsync(c->h_q, c->fargs.q, c->nq * 8, hipMemcpyDeviceToHost, c->stream)) != hipSuccess ||
            (e = hipMemcpyAsync(c->h_res, c->fargs.res, (size_t)count * 32, hipMemcpyDeviceToHost, c->stream)) !=
                hipSuccess ||
            (e = hipStreamSynchronize(c->stream)) != hipSuccess)
            return hip_fail(e, "batch results");
        if (p0->timing) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, p0->ev0, p0->ev1) == hipSuccess) {
                p0->kernel_ms += ms;
                p0->kernel_launches += 1;
            }
        }
        for (uint32_t i = 0; i < count; ++i) {
            const BatchSector &s = c->hs[i];
            bool fin = true;
            for (uint32_t k = 0; k < s.m * c->np; ++k) fin = fin && std::isfinite(c->h_q[s.q_off + k]);
            const double *r = c->h_res + 4 * i;
            out[i] = qmc_result{r[0], c->np == 2 ? r[1] : 0.0, r[2], c->np == 2 ? r[3] : 0.0, (int32_t)(c->np == 2), 0, 0.0};
            if (!fin) {
                out[i].mean_re = out[i].mean_im = out[i].err_re = out[i].err_im = NAN;
                any_nonfinite = true;
            }
        }
    }
    if (any_nonfinite) return fail(QMC_ENONFINITE, "a per-shift sum of some plan is not finite");
    return QMC_OK;
}

qmc_status qmc_batch_stats(uint64_t *out) {
    if (!out) return fail(QMC_EINVAL, "null argument");
    std::lock_guard<std::mutex> lock(g_batch_mu);
    std::copy(g_stats, g_stats + 4, out);
    return QMC_OK;
}

qmc_status qmc_batch_per_shift(uint32_t count, const qmc_plan_t *plans, double *const *per_shift) {
    if (!plans || !per_shift) return fail(QMC_EINVAL, "null argument");
    std::lock_guard<std::mutex> lock(g_batch_mu);
    for (auto &x : g_batch) {
        if (x->plans.size() != count || !std::equal(x->plans.begin(), x->plans.end(), plans)) continue;
        for (uint32_t i = 0; i < count; ++i)
            if (per_shift[i])
                std::memcpy(per_shift[i], x->h_q + x->hs[i].q_off, (size_t)x->hs[i].m * x->np * sizeof(double));
        return QMC_OK;
    }
    return fail(QMC_EINVAL, "no batch ran with these plans");
}

qmc_status qmc_batch_autotune(uint32_t count, const qmc_plan_t *plans, qmc_family family, const void *const *params,
                              qmc_batch_opts *best, double *best_ms) {
    if (count == 0) return fail(QMC_EINVAL, "count must be >= 1");
    if (!plans || !params || !best) return fail(QMC_EINVAL, "null argument");
    if (!plans[0]) return fail(QMC_EINVAL, "plan 0 is NULL");
    std::vector<qmc_result> out(count);
    qmc_plan_s *p0 = plans[0];
    const bool keep_timing = p0->timing;
    p0->timing = true;
    double best_t = INFINITY;
    qmc_batch_opts choice{1, 0, 8192, QMC_BATCH_DEFAULT};
    qmc_status st = QMC_OK;
    for (int32_t sched : {QMC_BATCH_DEFAULT, QMC_BATCH_PERSISTENT}) {
        for (uint32_t tp : {4096u, 8192u, 16384u, 32768u}) {
            const qmc_batch_opts o{1, 0, tp, sched};
            // one call per candidate: it captures the graph and launches it;
            // the events bracket the graph launch alone
            p0->kernel_ms = 0.0;
            p0->kernel_launches = 0;
            st = qmc_integrate_batch(count, plans, family, params, &o, out.data());
            if (st && st != QMC_ENONFINITE) break;
            const double t = p0->kernel_launches ? p0->kernel_ms / (double)p0->kernel_launches : INFINITY;
            if (st && st != QMC_ENONFINITE) break;
            if (t < best_t) {
                best_t = t;
                choice = o;
            }
        }
        if (st && st != QMC_ENONFINITE) break;
    }
    p0->timing = keep_timing;
    p0->kernel_ms = 0.0;
    p0->kernel_launches = 0;
    if (st && st != QMC_ENONFINITE) return st;
    *best = choice;
    if (best_ms) *best_ms = best_t;
    return QMC_OK;
}

}  // extern "C"
