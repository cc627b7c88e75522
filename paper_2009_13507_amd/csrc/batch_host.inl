// batch_host.inl -- batched imaginary-time stepping (included by ssgp.hip).
//
// A batch keeps one single-grid object per instance over its slice of the
// pool (source of the x-line tables, the one-instance-at-a-time path and the
// observables), the descriptor table and item lists of the batched kernels,
// and the HIP graphs of the chosen launch shape.
//
// Launch shapes: k > 0 is the persistent kernel with k workgroups per
// compute unit (every workgroup resident, device-wide barriers between the
// phases); -1 is one kernel launch per phase; -2 and -4 split the instances
// into 2 or 4 groups of about equal points, each group stepped by its own
// phase launches on a stream of its own (forked from the batch's stream and
// joined back), so that one group's x rows run beside another's y tiles.
// The grouped shapes are switched off (BATCH_GROUPS_ENABLED): a step call of
// a 64-instance batch ended in a segmentation fault of the host process
// while they were in use, with no cause found in this code.  All shapes run the same item functions, so
// the results do not depend on the shape.  The autotuner times every shape
// on a scratch copy of the pool at the first step call and keeps the
// fastest.  A run of n steps is replayed as graphs of 2^i steps (binary
// decomposition of n); a graph ends with the RENORM scale of its last step,
// which gives bitwise the same state as one longer run, since the next step
// would apply the same rounded product first.

static constexpr long long BATCH_SPIN_LIMIT = 1LL << 21;  // a second or more per barrier wait
static constexpr int BATCH_LOG2_PERSISTENT = 12;          // persistent graphs of up to 4096 steps
static constexpr int BATCH_LOG2_PHASED = 6;               // phase-launch graphs of up to 64 steps
static constexpr int BATCH_MAX_INSTANCES = 1 << 16;
// shapes -2 and -4 (8 groups measured slower than 4, 0.288 against 0.275 ms
// per complex128 C4 step: a process has 4 hardware queues by default, so
// 8 streams share them)
static constexpr int BATCH_GROUP_LEVELS = 2;
static constexpr int BATCH_MAX_GROUPS = 1 << BATCH_GROUP_LEVELS;

// The grouped shapes -2 and -4 are off until the cause of a host
// segmentation fault seen in a step call with them in use is found: the
// tuner does not time them and ssgp_batch_set_shape refuses them.
static constexpr bool BATCH_GROUPS_ENABLED = false;

// k for the grouped shape -2^k (1 <= k <= BATCH_GROUP_LEVELS), else 0.
static int batch_group_level(int shape) {
    for (int k = 1; k <= BATCH_GROUP_LEVELS; ++k)
        if (shape == -(1 << k)) return k;
    return 0;
}

// One group's item lists: x rows [xoff, xoff + nrows) (the first nrows2 by
// two wavefronts), y tiles [yoff, yoff + nyitems), instances [roff, roff + ninst).
struct BatchGroup {
    int xoff, nrows, nrows2, yoff, nyitems, roff, ninst;
};

template <typename R> struct BatchTabs {
    DevBuf inst;                // BatchInst<R>[n]
    std::vector<CNDev<R>> ly;   // y-line tables in the batched chunking
};

struct ssgp_batch_s {
    int n = 0, dtype = SSGP_C128, ncu = 1;
    void *pool = nullptr;
    size_t pool_bytes = 0;      // extent of the pool the instances use
    hipStream_t stream = nullptr, cap = nullptr;
    hipStream_t side[BATCH_MAX_GROUPS - 1] = {};  // the streams of groups 1, 2, ...
    hipEvent_t evf = nullptr, evj[BATCH_MAX_GROUPS - 1] = {};
    std::vector<BatchGroup> grouped[BATCH_GROUP_LEVELS];  // [k - 1]: the instances in 2^k groups (none if fewer instances)
    DevBuf gitems;                       // the groups' item lists, concatenated
    std::vector<ssgp_grid> grids;
    int nrows = 0, nrows2 = 0, nyitems = 0, ntiles = 0;
    DevBuf xitems, yitems, partials, renorm, bar;
    BatchTabs<double> t64;
    BatchTabs<float> t32;
    int occ = 0;                // resident persistent workgroups per compute unit
    int shape = 0;              // 0: choose at the next step call
    double shape_us = 0.0;      // measured microseconds per step of the shape in use (0 if not timed)
    std::vector<hipGraphExec_t> graphs;  // [log2 steps] for the shape in use
    void drop_graphs() {
        for (hipGraphExec_t &g : graphs)
            if (g) {
                (void)hipGraphExecDestroy(g);
                g = nullptr;
            }
    }
    ~ssgp_batch_s() {
        if (stream) (void)hipStreamSynchronize(stream);
        drop_graphs();
        for (ssgp_grid g : grids) ssgp_destroy(g);
        if (cap) (void)hipStreamDestroy(cap);
        for (int g = 0; g < BATCH_MAX_GROUPS - 1; ++g) {
            if (side[g]) (void)hipStreamDestroy(side[g]);
            if (evj[g]) (void)hipEventDestroy(evj[g]);
        }
        if (evf) (void)hipEventDestroy(evf);
    }
};

template <typename R> static BatchTabs<R> &btabs(ssgp_batch b);
template <> BatchTabs<double> &btabs<double>(ssgp_batch b) { return b->t64; }
template <> BatchTabs<float> &btabs<float>(ssgp_batch b) { return b->t32; }

// y chunk: smallest power of two with BATCH_THREADS/TX chunks covering ny
template <typename R> static int batch_y_chunk(int ny) {
    const int P = BATCH_THREADS / BatchTX<R>::v;
    return pow2_at_least((ny + P - 1) / P);
}

// Item lists of a set of instances (ids in instance order).  x rows and y
// tiles go the costliest first (rows by nx, tiles by ny), so that the
// round-robin assignment over the workgroups ends evenly; the rows by two
// wavefronts (x chunks of 8 points) come first.  y tiles go in blocks of 128
// list entries: the per-phase launch runs workgroup q on XCD q mod 8, so XCD
// k gets entries 16k .. 16k + 15 of the block, 16 adjacent column tiles of
// one instance and component (measured: 0.314 -> 0.303 ms per complex128
// step; 4 per XCD gave nothing, 8 nearly as much).  ri: the instances.
template <typename R>
static void batch_lists(const std::vector<BatchInst<R>> &host, std::vector<int> ids, std::vector<int> &xi, int &nrows2,
                        std::vector<int> &yi, std::vector<int> &ri) {
    ri = ids;
    std::stable_sort(ids.begin(), ids.end(), [&](int u, int v) { return host[u].nx > host[v].nx; });
    xi.clear();
    for (int i : ids)
        for (int r = 0; r < host[i].ny; ++r) xi.push_back((i << 10) | r);
    nrows2 = 0;
    if (batch_pair_rows<R>())
        for (int q : xi)
            if (host[q >> 10].Lx == 8) ++nrows2;
    std::stable_sort(ids.begin(), ids.end(), [&](int u, int v) { return host[u].ny > host[v].ny; });
    yi.clear();
    for (int i : ids)
        for (int j = 0; j < 3; ++j)
            for (int t = 0; t < host[i].ntiles; ++t) yi.push_back((i << 8) | (j << 6) | t);
    constexpr int G = 16, BLK = 8 * G;
    std::vector<int> p(yi);
    const int full = (int)yi.size() / BLK * BLK;
    for (int base = 0; base < full; base += BLK)
        for (int k = 0; k < 8; ++k)
            for (int m = 0; m < G; ++m) p[(size_t)(base + k + 8 * m)] = yi[(size_t)(base + G * k + m)];
    yi.swap(p);
}

template <typename R> static int batch_build(ssgp_batch b, const long long *offsets) {
    constexpr int TX = BatchTX<R>::v;
    const int P = BATCH_THREADS / TX;
    int maxlv = 0;
    while ((TX << maxlv) < 64) ++maxlv;
    BatchTabs<R> &T = btabs<R>(b);
    T.ly.resize(b->n);
    std::vector<BatchInst<R>> host(b->n);
    int tile_base = 0;
    for (int i = 0; i < b->n; ++i) {
        ssgp_grid g = b->grids[i];
        SSGP_TRY(build_tables<R>(g, MODE_IMAG));
        const XArgs<R> xa = x_args<R>(g, MODE_IMAG, nullptr, nullptr, g->p.omega, nullptr);
        const int Ly = batch_y_chunk<R>(g->ny);
        SSGP_TRY(upload_cn<R>(T.ly[i], cn_tables(g->ny, g->dy, cn_s(MODE_IMAG, g->p.dt), Ly, P, maxlv), g->ny, Ly, P,
                              b->stream));
        BatchInst<R> &I = host[i];
        I = BatchInst<R>{};
        I.off = offsets[i];
        I.nx = g->nx;
        I.ny = g->ny;
        I.Lx = x_chunk(g->nx);
        I.Ly = Ly;
        I.ntiles = (g->nx + TX - 1) / TX;
        I.tile_base = tile_base;
        tile_base += I.ntiles;
        I.dx = xa.dx;
        I.dy = xa.dy;
        I.x0 = xa.x0;
        I.y0 = xa.y0;
        I.m = xa.m;
        I.lx = tables<R>(g).x[MODE_IMAG].coef();
        I.lv4 = cn_tables(g->nx, g->dx, cn_s(MODE_IMAG, g->p.dt), 4, 128, 6).levels;
        I.ly = T.ly[i].coef();
        I.rdx = xa.rdiag;
        I.rdy = T.ly[i].rdiag;
        for (int q = 0; q < 9; ++q) I.qx[q] = xa.qx[q];
        I.qxmask = xa.qxmask;
        if (!so_pattern_of(I.qx, I.qxmask, I.sopat, I.qa, I.qb) || I.sopat == 2)
            return fail(SSGP_EINVAL, "instance %d: SO coefficients of an unexpected pattern", i);
        I.sp = renorm_spec(*g);
    }
    b->ntiles = tile_base;
    SSGP_TRY(T.inst.ensure(sizeof(BatchInst<R>) * b->n));
    HIP_TRY(hipMemcpyAsync(T.inst.p, host.data(), sizeof(BatchInst<R>) * b->n, hipMemcpyHostToDevice, b->stream));

    std::vector<int> all(b->n);
    for (int i = 0; i < b->n; ++i) all[i] = i;
    std::vector<int> xi, yi, ri;
    int nrows2 = 0;
    batch_lists<R>(host, all, xi, nrows2, yi, ri);
    b->nrows = (int)xi.size();
    b->nrows2 = nrows2;
    b->nyitems = (int)yi.size();
    SSGP_TRY(b->xitems.ensure(sizeof(int) * xi.size()));
    SSGP_TRY(b->yitems.ensure(sizeof(int) * yi.size()));
    HIP_TRY(hipMemcpyAsync(b->xitems.p, xi.data(), sizeof(int) * xi.size(), hipMemcpyHostToDevice, b->stream));
    HIP_TRY(hipMemcpyAsync(b->yitems.p, yi.data(), sizeof(int) * yi.size(), hipMemcpyHostToDevice, b->stream));

    // the instances in 2 and 4 groups: by points, largest first, each to the
    // group with the fewest points so far (the first such group on ties)
    std::vector<int> gl;
    for (int k = 1; k <= BATCH_GROUP_LEVELS; ++k) {
        const int G = 1 << k;
        b->grouped[k - 1].clear();
        if (G > b->n) continue;
        std::vector<int> bysize(all);
        std::stable_sort(bysize.begin(), bysize.end(), [&](int u, int v) {
            return (long long)host[u].nx * host[u].ny > (long long)host[v].nx * host[v].ny;
        });
        std::vector<std::vector<int>> members(G);
        std::vector<long long> load(G, 0);
        for (int i : bysize) {
            int g = 0;
            for (int h = 1; h < G; ++h)
                if (load[h] < load[g]) g = h;
            members[g].push_back(i);
            load[g] += (long long)host[i].nx * host[i].ny;
        }
        for (int g = 0; g < G; ++g) {
            std::sort(members[g].begin(), members[g].end());
            std::vector<int> gx, gy, gr;
            int g2 = 0;
            batch_lists<R>(host, members[g], gx, g2, gy, gr);
            BatchGroup bg{};
            bg.xoff = (int)gl.size();
            bg.nrows = (int)gx.size();
            bg.nrows2 = g2;
            gl.insert(gl.end(), gx.begin(), gx.end());
            bg.yoff = (int)gl.size();
            bg.nyitems = (int)gy.size();
            gl.insert(gl.end(), gy.begin(), gy.end());
            bg.roff = (int)gl.size();
            bg.ninst = (int)gr.size();
            gl.insert(gl.end(), gr.begin(), gr.end());
            b->grouped[k - 1].push_back(bg);
        }
    }
    if (!gl.empty()) {
        SSGP_TRY(b->gitems.ensure(sizeof(int) * gl.size()));
        HIP_TRY(hipMemcpyAsync(b->gitems.p, gl.data(), sizeof(int) * gl.size(), hipMemcpyHostToDevice, b->stream));
    }
    SSGP_TRY(b->partials.ensure(sizeof(double) * 3 * b->ntiles));
    SSGP_TRY(b->renorm.ensure(sizeof(double) * 8 * b->n));
    SSGP_TRY(b->bar.ensure(sizeof(unsigned) * 4));
    HIP_TRY(hipMemsetAsync(b->renorm.p, 0, sizeof(double) * 8 * b->n, b->stream));
    HIP_TRY(hipMemsetAsync(b->bar.p, 0, sizeof(unsigned) * 4, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));  // the host vectors above go out of scope
    HIP_TRY(batch_occupancy<R>(&b->occ));
    if (b->occ < 1) return fail(SSGP_EDEVICE, "the batched kernel does not fit on a compute unit");
    return SSGP_OK;
}

template <typename R> static BatchArgs<R> batch_args(ssgp_batch b, void *pool, int nsteps) {
    BatchArgs<R> a{};
    a.pool = static_cast<cx<R> *>(pool);
    a.inst = btabs<R>(b).inst.template as<BatchInst<R>>();
    a.x_items = b->xitems.as<int>();
    a.y_items = b->yitems.as<int>();
    a.nrows = b->nrows;
    a.nrows2 = b->nrows2;
    a.nyitems = b->nyitems;
    a.partials = b->partials.as<double>();
    a.renorm = b->renorm.as<double>();
    a.ninst = b->n;
    a.bar = b->bar.as<unsigned>();
    a.nsteps = nsteps;
    a.spin_limit = BATCH_SPIN_LIMIT;
    return a;
}

// The arguments of one group's phase launches: its item lists.
template <typename R>
static BatchArgs<R> batch_args_group(ssgp_batch b, void *pool, int nsteps, const BatchGroup &g) {
    BatchArgs<R> a = batch_args<R>(b, pool, nsteps);
    const int *L = b->gitems.as<int>();
    a.x_items = L + g.xoff;
    a.nrows = g.nrows;
    a.nrows2 = g.nrows2;
    a.y_items = L + g.yoff;
    a.nyitems = g.nyitems;
    a.r_items = L + g.roff;
    a.ninst = g.ninst;
    return a;
}

// nsteps steps of the rows, tiles and instances in `a` by one launch per phase.
template <typename R> static int batch_enqueue_phases(hipStream_t st, const BatchArgs<R> &a, int nsteps) {
    for (int s = 0; s < nsteps; ++s) {
        LAUNCH_TRY(launch_batch_phase<R>(st, a, BATCH_PHASE_X, s > 0 ? 1 : 0));
        LAUNCH_TRY(launch_batch_phase<R>(st, a, BATCH_PHASE_Y, 0));
        LAUNCH_TRY(launch_batch_phase<R>(st, a, BATCH_PHASE_R, 0));
    }
    LAUNCH_TRY(launch_batch_phase<R>(st, a, BATCH_PHASE_SCALE, 0));
    return SSGP_OK;
}

// Enqueues nsteps steps of the pool at `pool` in launch shape `shape`.
template <typename R> static int batch_enqueue(ssgp_batch b, hipStream_t st, void *pool, int nsteps, int shape) {
    if (nsteps <= 0) return SSGP_OK;
    if (shape > 0) {
        LAUNCH_TRY(launch_batch_reset(st, b->bar.as<unsigned>()));
        LAUNCH_TRY(launch_batch_persistent<R>(st, batch_args<R>(b, pool, nsteps), shape * b->ncu));
        return SSGP_OK;
    }
    if (shape == -1) return batch_enqueue_phases<R>(st, batch_args<R>(b, pool, nsteps), nsteps);
    // groups: group 0 on st, group g on side[g - 1], forked from st and
    // joined back into it (under stream capture: parallel branches)
    const int lv = batch_group_level(shape);
    if (lv == 0) return fail(SSGP_EINVAL, "unknown launch shape %d", shape);
    const std::vector<BatchGroup> &gs = b->grouped[lv - 1];
    if (gs.empty()) return fail(SSGP_EINVAL, "launch shape %d needs at least %d instances", shape, -shape);
    HIP_TRY(hipEventRecord(b->evf, st));
    for (size_t g = 1; g < gs.size(); ++g) HIP_TRY(hipStreamWaitEvent(b->side[g - 1], b->evf, 0));
    int rc = SSGP_OK;
    for (size_t g = 0; g < gs.size() && rc == SSGP_OK; ++g)
        rc = batch_enqueue_phases<R>(g == 0 ? st : b->side[g - 1], batch_args_group<R>(b, pool, nsteps, gs[g]), nsteps);
    // joined even after a failed launch, so that no side stream is left forked
    for (size_t g = 1; g < gs.size(); ++g) {
        if (hipEventRecord(b->evj[g - 1], b->side[g - 1]) != hipSuccess ||
            hipStreamWaitEvent(st, b->evj[g - 1], 0) != hipSuccess)
            if (rc == SSGP_OK) rc = fail(SSGP_EDEVICE, "joining the group streams failed");
    }
    return rc;
}

// nsteps steps of the pool at `pool` in launch shape `shape`, captured and
// instantiated as a graph.
template <typename R>
static int batch_capture(ssgp_batch b, void *pool, int nsteps, int shape, hipGraphExec_t *out) {
    *out = nullptr;
    HIP_TRY(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    const int rc = batch_enqueue<R>(b, b->cap, pool, nsteps, shape);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(b->cap, &graph);
    if (rc != SSGP_OK || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        SSGP_TRY(rc);
        return fail(SSGP_EDEVICE, "hipStreamEndCapture failed: %s", hipGetErrorString(e));
    }
    const hipError_t e2 = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e2 != hipSuccess) {
        *out = nullptr;
        return fail(SSGP_EDEVICE, "hipGraphInstantiate failed: %s", hipGetErrorString(e2));
    }
    return SSGP_OK;
}

// Times every launch shape on a scratch copy of the pool, as the graph
// replays it will run as (eager launches would charge the grouped shapes
// their host launch time): the fastest of 3 replays of 8 steps after a
// warm-up replay.  Keeps the fastest shape.
template <typename R> static int batch_tune(ssgp_batch b) {
    DevBuf scratch;
    SSGP_TRY(scratch.ensure(b->pool_bytes));
    HIP_TRY(hipMemcpyAsync(scratch.p, b->pool, b->pool_bytes, hipMemcpyDeviceToDevice, b->stream));
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(SSGP_EDEVICE, "hipEventCreate failed");
    }
    std::vector<int> shapes = {-1};
    if (BATCH_GROUPS_ENABLED)
        for (int k = 1; k <= BATCH_GROUP_LEVELS; ++k)
            if (!b->grouped[k - 1].empty()) shapes.push_back(-(1 << k));
    for (int k = 1; k <= b->occ; ++k) shapes.push_back(k);
    const int steps = 8, reps = 3;
    int best = 0;
    double best_us = 0.0;
    int rc = SSGP_OK;
    for (int shape : shapes) {
        double t_min = 1e300;
        hipGraphExec_t exec = nullptr;
        rc = batch_capture<R>(b, scratch.p, steps, shape, &exec);
        for (int r = 0; r <= reps && rc == SSGP_OK; ++r) {  // r = 0 warms up
            if (hipEventRecord(e0, b->stream) != hipSuccess) rc = fail(SSGP_EDEVICE, "hipEventRecord failed");
            if (rc == SSGP_OK && hipGraphLaunch(exec, b->stream) != hipSuccess)
                rc = fail(SSGP_EDEVICE, "hipGraphLaunch failed");
            if (rc == SSGP_OK && hipEventRecord(e1, b->stream) != hipSuccess)
                rc = fail(SSGP_EDEVICE, "hipEventRecord failed");
            if (rc == SSGP_OK && hipEventSynchronize(e1) != hipSuccess)
                rc = fail(SSGP_EDEVICE, "hipEventSynchronize failed");
            float ms = 0.f;
            if (rc == SSGP_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                rc = fail(SSGP_EDEVICE, "hipEventElapsedTime failed");
            if (rc == SSGP_OK && r > 0) t_min = std::min(t_min, 1e3 * ms / steps);
        }
        if (exec) (void)hipGraphExecDestroy(exec);
        if (rc != SSGP_OK) break;
        if (best == 0 || t_min < best_us) {
            best = shape;
            best_us = t_min;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    SSGP_TRY(rc);
    unsigned flag[4] = {0, 0, 0, 0};
    HIP_TRY(hipMemcpy(flag, b->bar.p, sizeof flag, hipMemcpyDeviceToHost));
    if (flag[2] != 0u || flag[3] != 0u)
        return fail(SSGP_EDEVICE, "a device-wide barrier of the batched kernel timed out while tuning");
    b->shape = best;
    b->shape_us = best_us;
    return SSGP_OK;
}

template <typename R> static int batch_graph(ssgp_batch b, int lg, hipGraphExec_t *out) {
    if ((int)b->graphs.size() <= lg) b->graphs.resize(lg + 1, nullptr);
    if (!b->graphs[lg]) SSGP_TRY(batch_capture<R>(b, b->pool, 1 << lg, b->shape, &b->graphs[lg]));
    *out = b->graphs[lg];
    return SSGP_OK;
}

template <typename R> static int batch_step_t(ssgp_batch b, int nsteps) {
    if (nsteps == 0) return SSGP_OK;
    if (b->shape == 0) SSGP_TRY(batch_tune<R>(b));
    const int maxlg = b->shape > 0 ? BATCH_LOG2_PERSISTENT : BATCH_LOG2_PHASED;
    int rem = nsteps;
    for (int lg = maxlg; lg >= 0; --lg) {
        while (rem >= (1 << lg)) {
            hipGraphExec_t g = nullptr;
            SSGP_TRY(batch_graph<R>(b, lg, &g));
            HIP_TRY(hipGraphLaunch(g, b->stream));
            rem -= 1 << lg;
        }
    }
    return SSGP_OK;
}

// ---------------------------------------------------------------- ABI ---
extern "C" int ssgp_create_batch(int n, const int *nx, const int *ny, const double *dx, const ssgp_params *p,
                                 int dtype, void *pool_dev, const long long *offsets, void *hip_stream,
                                 ssgp_batch *out) {
    if (!out) return fail(SSGP_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || n > BATCH_MAX_INSTANCES) return fail(SSGP_EINVAL, "n must be in [1, %d]", BATCH_MAX_INSTANCES);
    if (!nx || !ny || !dx || !p || !offsets || !pool_dev) return fail(SSGP_EINVAL, "NULL argument");
    if (dtype != SSGP_C128 && dtype != SSGP_C64) return fail(SSGP_EINVAL, "unknown dtype %d", dtype);
    std::vector<std::pair<long long, long long>> spans(n);
    for (int i = 0; i < n; ++i) {
        if (nx[i] < 1 || nx[i] > BATCH_MAX_N || ny[i] < 1 || ny[i] > BATCH_MAX_N)
            return fail(SSGP_EINVAL, "instance %d: nx and ny must be in [1, %d]", i, BATCH_MAX_N);
        if (!(dx[i] > 0) || !std::isfinite(dx[i])) return fail(SSGP_EINVAL, "instance %d: dx must be positive", i);
        if (offsets[i] < 0) return fail(SSGP_EINVAL, "instance %d: negative offset", i);
        if (so_y_terms(p[i].so) && p[i].gamma != 0.0)
            return fail(SSGP_EINVAL, "instance %d: y-dependent SO forms are not supported in batched mode", i);
        spans[i] = {offsets[i], offsets[i] + 3LL * nx[i] * ny[i]};
    }
    std::sort(spans.begin(), spans.end());
    for (int i = 1; i < n; ++i)
        if (spans[i].first < spans[i - 1].second) return fail(SSGP_EINVAL, "instance states overlap in the pool");
    ssgp_batch b = new (std::nothrow) ssgp_batch_s();
    if (!b) return fail(SSGP_ENOMEM, "host allocation failed");
    b->n = n;
    b->dtype = dtype;
    b->pool = pool_dev;
    b->pool_bytes = (size_t)spans[n - 1].second * elem_bytes(dtype);
    b->stream = static_cast<hipStream_t>(hip_stream);
    int rc = SSGP_OK;
    for (int i = 0; i < n && rc == SSGP_OK; ++i) {
        ssgp_grid g = nullptr;
        rc = ssgp_create_grid(2, nx[i], ny[i], dx[i], dx[i], dtype,
                              static_cast<char *>(pool_dev) + offsets[i] * (long long)elem_bytes(dtype), hip_stream, &g);
        if (rc == SSGP_OK) {
            b->grids.push_back(g);
            rc = ssgp_set_params(g, &p[i]);
            if (rc != SSGP_OK) {
                const std::string m = g_err;
                rc = fail(rc, "instance %d: %s", i, m.c_str());
            }
        }
    }
    if (rc == SSGP_OK) b->ncu = b->grids[0]->ncu;
    if (rc == SSGP_OK && hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess)
        rc = fail(SSGP_EDEVICE, "hipStreamCreateWithFlags failed");
    for (int g = 0; g < BATCH_MAX_GROUPS - 1 && rc == SSGP_OK; ++g)
        if (hipStreamCreateWithFlags(&b->side[g], hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&b->evj[g], hipEventDisableTiming) != hipSuccess)
            rc = fail(SSGP_EDEVICE, "creating the group streams failed");
    if (rc == SSGP_OK && hipEventCreateWithFlags(&b->evf, hipEventDisableTiming) != hipSuccess)
        rc = fail(SSGP_EDEVICE, "hipEventCreateWithFlags failed");
    if (rc == SSGP_OK) rc = dtype == SSGP_C128 ? batch_build<double>(b, offsets) : batch_build<float>(b, offsets);
    if (rc != SSGP_OK) {
        delete b;
        return rc;
    }
    *out = b;
    return SSGP_OK;
}

extern "C" int ssgp_batch_step_imag(ssgp_batch b, int nsteps) {
    if (!b) return fail(SSGP_EINVAL, "batch is NULL");
    if (nsteps < 0) return fail(SSGP_EINVAL, "nsteps < 0");
    return b->dtype == SSGP_C128 ? batch_step_t<double>(b, nsteps) : batch_step_t<float>(b, nsteps);
}

extern "C" int ssgp_batch_step_imag_serial(ssgp_batch b, int nsteps) {
    if (!b) return fail(SSGP_EINVAL, "batch is NULL");
    if (nsteps < 0) return fail(SSGP_EINVAL, "nsteps < 0");
    for (ssgp_grid g : b->grids) SSGP_TRY(ssgp_step_imag(g, nsteps));
    return SSGP_OK;
}

extern "C" int ssgp_batch_set_shape(ssgp_batch b, int shape) {
    if (!b) return fail(SSGP_EINVAL, "batch is NULL");
    const int lv = batch_group_level(shape);
    if ((shape < -1 && lv == 0) || shape > b->occ)
        return fail(SSGP_EINVAL, "shape must be -4, -2, -1, 0 or a workgroup count in [1, %d] per compute unit",
                    b->occ);
    if (lv > 0 && !BATCH_GROUPS_ENABLED) return fail(SSGP_EINVAL, "the grouped launch shapes are switched off");
    if (lv > 0 && b->grouped[lv - 1].empty())
        return fail(SSGP_EINVAL, "launch shape %d needs at least %d instances", shape, -shape);
    if (shape != b->shape) {
        HIP_TRY(hipStreamSynchronize(b->stream));
        b->drop_graphs();
        b->shape = shape;
        b->shape_us = 0.0;
    }
    return SSGP_OK;
}

extern "C" int ssgp_batch_info(ssgp_batch b, double *out) {
    if (!b || !out) return fail(SSGP_EINVAL, "NULL argument");
    out[0] = b->shape;
    out[1] = b->shape > 0 ? (double)b->shape * b->ncu : 0.0;
    out[2] = b->occ;
    out[3] = b->shape_us;
    out[4] = b->nrows;
    out[5] = b->nyitems;
    return SSGP_OK;
}

extern "C" int ssgp_batch_sync(ssgp_batch b) {
    if (!b) return fail(SSGP_EINVAL, "batch is NULL");
    HIP_TRY(hipStreamSynchronize(b->stream));
    unsigned flag[4] = {0, 0, 0, 0};
    HIP_TRY(hipMemcpy(flag, b->bar.p, sizeof flag, hipMemcpyDeviceToHost));
    if (flag[2] != 0u || flag[3] != 0u) {
        HIP_TRY(hipMemsetAsync(b->bar.p, 0, sizeof(unsigned) * 4, b->stream));
        HIP_TRY(hipStreamSynchronize(b->stream));
        return fail(SSGP_EDEVICE, "a device-wide barrier of the batched kernel timed out; the batch state is invalid");
    }
    return SSGP_OK;
}

extern "C" int ssgp_batch_observables(ssgp_batch b, ssgp_obs *out) {
    if (!b || !out) return fail(SSGP_EINVAL, "NULL argument");
    SSGP_TRY(ssgp_batch_sync(b));
    int rc = SSGP_OK;
    for (int i = 0; i < b->n; ++i) {
        const int r = ssgp_observables(b->grids[i], &out[i]);
        if (r == SSGP_ENONFINITE && rc == SSGP_OK) rc = fail(r, "instance %d holds NaN or Inf", i);
        else if (r != SSGP_OK && r != SSGP_ENONFINITE) return r;
    }
    return rc;
}

extern "C" int ssgp_destroy_batch(ssgp_batch b) {
    delete b;
    return SSGP_OK;
}
