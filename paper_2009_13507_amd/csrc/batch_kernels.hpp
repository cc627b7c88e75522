// batch_kernels.hpp -- many independent 2D grids (uneven sizes and
// parameters) advanced together in imaginary time.
//
// Per step, over all instances of the batch:
//   X phase, items (instance, row): RENORM scale of the previous step,
//      CALCNU, HERM, SO, the Crank-Nicolson right-hand side and the x-line
//      solve of one row, all by one wavefront (batch_xrow_wave: each lane
//      owns L consecutive points of the three components, no barrier);
//   Y phase, items (instance, component, tile of TX columns): the y-line
//      solve (chunks in registers, chunk scans across the workgroup) and the
//      tile's sum of |psi|^2;
//   R phase, items (instance): the fixed-order sum of the instance's tile
//      sums and its RENORM factors (App. A, Eq. (DJ) or (DJ2)), which the
//      next X phase applies.
// After the last step a scale phase applies the last RENORM factors, so the
// state is normalised on return.
//
// The phases run either as one persistent kernel with device-wide barriers
// between them, or as one kernel launch per phase; both execute the same
// item functions with the same arithmetic, so their results are identical.
//
// Barrier: arrivals are counted on a global word and waiters are released by
// a generation word (vector atomics at agent scope; one agent-scope release
// fence per workgroup before its arrival and one acquire fence after the
// wait, so that the state written before the barrier is visible after it on
// every XCD).  Every wait is bounded: a workgroup whose wait exceeds the
// spin budget raises a stop word and leaves; every other workgroup sees the
// word at its next barrier and leaves too, so the grid always drains.
#pragma once
#include "step_kernels.hpp"

namespace ssgp {

constexpr int BATCH_THREADS = 256;
constexpr int BATCH_MAX_LX = 8;  // x chunk: rows of up to 64 * 8 = 512 points
constexpr int BATCH_MAX_N = 512;

// y tile width: one 128-byte line of each row per tile
template <typename R> struct BatchTX;
template <> struct BatchTX<double> { static constexpr int v = 8; };
template <> struct BatchTX<float> { static constexpr int v = 16; };

template <typename R> struct BatchInst {
    long long off;             // first element of the instance's state in the pool
    int nx, ny, Lx, Ly;        // x chunk (64 chunks per row), y chunk (BATCH_THREADS/TX chunks per column)
    int ntiles;                // ceil(nx / TX)
    int tile_base;             // index of the instance's first tile in the partials array
    R dx, dy, x0, y0;
    Model<R> m;
    LineCoef<R> lx, ly;        // elimination coefficients of the x and y lines
    int lv4;                   // scan levels of x lines in chunks of 4 points (two-wavefront rows)
    cx<R> rdx, rdy;            // diagonal of (I - sT)/o of x and y (off-diagonal -1)
    cx<R> qx[9];               // SO: psi'_j += sum_j' qx[j][j'] (psi_j'(i+1) - psi_j'(i-1))
    unsigned qxmask;
    int sopat;                 // what the row kernels read of qx (as XArgs::sopat): 1 neighbouring
    cx<R> qa, qb;              // components (qa = qx[0][1] = qx[1][2], qb = qx[1][0] = qx[2][1]), 0 none
    RenormSpec sp;
};

// SO update of a row's L consecutive points from the two coefficients of
// the neighbouring-component pattern (each component's terms in the order
// j' = 0, 1, 2); vb, va: the values just before and after the points.
template <typename R, int L>
__device__ __forceinline__ void so_neighbours(cx<R> (&u)[3][L], const cx<R> (&v)[3][L], const cx<R> (&vb)[3],
                                              const cx<R> (&va)[3], cx<R> qa, cx<R> qb) {
#pragma unroll
    for (int t = 0; t < L; ++t) {
        cx<R> d[3];
#pragma unroll
        for (int jp = 0; jp < 3; ++jp) {
            const cx<R> pv = t > 0 ? v[jp][t > 0 ? t - 1 : 0] : vb[jp];
            const cx<R> nv = t + 1 < L ? v[jp][t + 1 < L ? t + 1 : 0] : va[jp];
            d[jp] = nv - pv;
        }
        u[0][t] = cfma(qa, d[1], u[0][t]);
        u[1][t] = cfma(qa, d[2], cfma(qb, d[0], u[1][t]));
        u[2][t] = cfma(qb, d[1], u[2][t]);
    }
}

template <typename R> struct BatchArgs {
    cx<R> *pool;
    const BatchInst<R> *inst;
    const int *x_items;        // (instance << 10) | row
    const int *y_items;        // (instance << 8) | (component << 6) | tile
    int nrows, nyitems;
    int nrows2;                // x_items[0, nrows2): rows by two wavefronts (batch_xrow_pair)
    double *partials;          // [total tiles][3] tile sums of |psi|^2
    double *renorm;            // [instances][8]: d[3], N[3], fallback
    int ninst;
    const int *r_items;        // instances of the R phase (nullptr: 0 .. ninst - 1)
    unsigned *bar;             // [0] arrivals, [1] generation, [2] stop, [3] sticky timeout flag
    int nsteps;
    long long spin_limit;
};

__device__ __forceinline__ double coherent_load(const double *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Device-wide barrier; returns false when the grid must stop.  Every
// thread's stores are complete (workgroup-scope release) before the
// workgroup barrier; thread 0 then makes them visible to the other XCDs
// (agent-scope release fence) and arrives, waits on the generation word with
// relaxed loads (no cache invalidation per poll) and takes one agent-scope
// acquire fence when it changes, which the workgroup barrier passes on.
__device__ __forceinline__ bool grid_sync(unsigned *bar, long long spin_limit) {
    __shared__ int stop;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const unsigned gen = __hip_atomic_load(bar + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned arrived = __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (arrived == gridDim.x - 1) {
            __hip_atomic_store(bar, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(bar + 1, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            long long spins = 0;
            while (__hip_atomic_load(bar + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                if (__hip_atomic_load(bar + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) break;
                if (++spins > spin_limit) {
                    __hip_atomic_store(bar + 2, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        stop = __hip_atomic_load(bar + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
    }
    __syncthreads();
    return !stop;
}

// Shared memory of one workgroup.
template <typename R> struct BatchSmem {
    cx<R> line[64 * BATCH_MAX_LX + 64 + 1];  // the y pivot head
    cx<R> scA[2][4][BatchTX<R>::v], scB[2][4][BatchTX<R>::v];
    double red[3][BATCH_THREADS];
};

// One x row of one instance by one wavefront (rows of at most 64 L points).
// Lane l owns the L consecutive points l L .. l L + L - 1 of all three
// components from the loads to the stores: RENORM scale, CALCNU + HERM, the
// SO update and the right-hand side in registers (the values just outside a
// lane's points come from the neighbouring lanes by DPP rotations; the row
// ends are the zero ghosts), then the three lines' chunk eliminations, one
// affine-map scan per sweep within the wavefront and the carry fix-ups (the
// same elimination as the 4-wavefront row code: 64 chunks of L points), and
// coalesced stores through the wavefront's own LDS line.  No barrier: the
// wavefronts of a workgroup work on different rows.
template <typename R, int L> constexpr int bx_line_slots() { return 64 * L + 64; }
template <typename R, int L>
__device__ __forceinline__ void batch_xrow_wave(const BatchInst<R> &I, cx<R> *psi, int row, const double *dscale,
                                                cx<R> *line) {
    const int lane = threadIdx.x & 63;
    const int nx = I.nx;
    const long long plane = (long long)nx * I.ny;
    const int i0 = lane * L;
    const int len = max(0, min(L, nx - i0));
    cx<R> *rowp = psi + (long long)row * nx;
    cx<R> v[3][L];
#pragma unroll
    for (int t = 0; t < L; ++t)
#pragma unroll
        for (int j = 0; j < 3; ++j) v[j][t] = t < len ? rowp[j * plane + i0 + t] : czero<R>();
    {
        R d0 = R(1), d1 = R(1), d2 = R(1);
        if (dscale) {
            d0 = R(coherent_load(dscale + 0));
            d1 = R(coherent_load(dscale + 1));
            d2 = R(coherent_load(dscale + 2));
        }
        const R yv = I.y0 + R(row) * I.dy;
        const R vy = R(0.5) * I.m.kappa2 * yv * yv;
#pragma unroll
        for (int t = 0; t < L; ++t) {
            if (t < len) {
                if (dscale) {
                    v[0][t] = d0 * v[0][t];
                    v[1][t] = d1 * v[1][t];
                    v[2][t] = d2 * v[2][t];
                }
                const R xv = I.x0 + R(i0 + t) * I.dx;
                pointwise(v[0][t], v[1][t], v[2][t], R(0.5) * xv * xv + vy, I.m);
            }
        }
    }
    // values just outside this lane's points (zero beyond the row's ends)
    auto outer = [&](const cx<R> (&x)[L], cx<R> &before, cx<R> &after) {
        before = ror1(x[L - 1]);
        after = rol1(x[0]);
        if (lane == 0) before = czero<R>();
        if (lane == 63) after = czero<R>();
    };
    // SO update u = v + q (v(i+1) - v(i-1))
    cx<R> u[3][L];
    {
        cx<R> vb[3], va[3];
#pragma unroll
        for (int jp = 0; jp < 3; ++jp) outer(v[jp], vb[jp], va[jp]);
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int t = 0; t < L; ++t) u[j][t] = v[j][t];
        if (I.sopat) so_neighbours<R, L>(u, v, vb, va, I.qa, I.qb);
#pragma unroll
        for (int t = 0; t < L; ++t)
            if (t >= len)
#pragma unroll
                for (int j = 0; j < 3; ++j) u[j][t] = czero<R>();
    }
    // right-hand side (I - sT) u / o
    cx<R> r[3][L];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        cx<R> ub, ua;
        outer(u[j], ub, ua);
#pragma unroll
        for (int t = 0; t < L; ++t) {
            const cx<R> pu = t > 0 ? u[j][t > 0 ? t - 1 : 0] : ub;
            const cx<R> nu = t + 1 < L ? u[j][t + 1 < L ? t + 1 : 0] : ua;
            r[j][t] = t < len ? cn_rhs(I.rdx, u[j][t], pu + nu) : czero<R>();
        }
    }
    // the three lines: chunk eliminations, scans within the wavefront, fix-ups
    const ChunkCoef<R, L, 0> cpl(I.lx, i0);
    const cx<R> Ak = I.lx.chunkA[lane];
    cx<R> A[3], B[3], carry[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        A[j] = Ak;
        B[j] = fwd_local<R, L>(r[j], len, cpl);
    }
    wave_scan_up3<R>(A, B, I.lx.levels);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        carry[j] = shfl_up(B[j], 1);
        if (lane == 0) carry[j] = czero<R>();
    }
    fwd_fix3<R, L, 0>(r, len, cpl, carry);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        A[j] = Ak;
        B[j] = bwd_local<R, L>(r[j], len, cpl);
    }
    wave_scan_down3<R>(A, B, I.lx.levels);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        carry[j] = shfl_down(B[j], 1);
        if (lane == 63) carry[j] = czero<R>();
    }
    bwd_fix3<R, L, 0>(r, len, cpl, carry);
    // coalesced stores (store k of lane l: point 64 k + l)
    if constexpr (L == 1) {
#pragma unroll
        for (int j = 0; j < 3; ++j)
            if (len > 0) rowp[j * plane + lane] = r[j][0];
    } else {
        cx<R> c0[L], c1[L], c2[L];
        wave_exchange<R, L>(line, lane, r[0], c0);
        wave_exchange<R, L>(line, lane, r[1], c1);
        wave_exchange<R, L>(line, lane, r[2], c2);
#pragma unroll
        for (int k = 0; k < L; ++k) {
            const int i = 64 * k + lane;
            if (i < nx) {
                put2(rowp + i, c0[k]);
                put2(rowp + plane + i, c1[k]);
                put2(rowp + 2 * plane + i, c2[k]);
            }
        }
    }
}

// Rows by two wavefronts (in double precision the rows of 257..512 points,
// whose one-wavefront form needs the registers of two).  Thread t of the
// pair owns the 4 consecutive points 4 t .. 4 t + 3: as batch_xrow_wave, with
// the values across the two wavefronts' boundary and the chunk maps of the
// first (forward) or second (backward) wavefront passed through LDS; the line
// is eliminated in 128 chunks of 4 points, each lane's chunk product formed
// from its pivots.  Every thread of the workgroup calls it the same number of
// times (it holds barriers); `active` is false for a pair with no row.
template <typename R> constexpr bool batch_pair_rows() { return sizeof(R) == 8; }

template <typename R> struct PairSmem {
    cx<R> E[2][2][2][3];           // [round][wave][end][component]
    cx<R> scA[2][2][3], scB[2][2][3];  // [sweep][wave][component]
};

template <typename R>
__device__ __forceinline__ void batch_xrow_pair(const BatchInst<R> &I, cx<R> *psi, int row, const double *dscale,
                                                cx<R> *line, PairSmem<R> &P, bool active) {
    constexpr int L = 4;
    const int tid = threadIdx.x & 127, w = tid >> 6, lane = tid & 63;
    const int nx = active ? I.nx : 0;
    const long long plane = active ? (long long)nx * I.ny : 0;
    const int i0 = tid * L;
    const int len = max(0, min(L, nx - i0));
    cx<R> *rowp = active ? psi + (long long)row * nx : psi;
    cx<R> v[3][L];
#pragma unroll
    for (int t = 0; t < L; ++t)
#pragma unroll
        for (int j = 0; j < 3; ++j) v[j][t] = t < len ? rowp[j * plane + i0 + t] : czero<R>();
    if (active) {
        R d0 = R(1), d1 = R(1), d2 = R(1);
        if (dscale) {
            d0 = R(coherent_load(dscale + 0));
            d1 = R(coherent_load(dscale + 1));
            d2 = R(coherent_load(dscale + 2));
        }
        const R yv = I.y0 + R(row) * I.dy;
        const R vy = R(0.5) * I.m.kappa2 * yv * yv;
#pragma unroll
        for (int t = 0; t < L; ++t) {
            if (t < len) {
                if (dscale) {
                    v[0][t] = d0 * v[0][t];
                    v[1][t] = d1 * v[1][t];
                    v[2][t] = d2 * v[2][t];
                }
                const R xv = I.x0 + R(i0 + t) * I.dx;
                pointwise(v[0][t], v[1][t], v[2][t], R(0.5) * xv * xv + vy, I.m);
            }
        }
    }
    auto publish = [&](const cx<R> (&x)[3][L], int round) {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            if (lane == 0) P.E[round][w][0][j] = x[j][0];
            if (lane == 63) P.E[round][w][1][j] = x[j][L - 1];
        }
    };
    auto outer = [&](const cx<R> (&x)[L], int round, int j, cx<R> &before, cx<R> &after) {
        before = ror1(x[L - 1]);
        after = rol1(x[0]);
        if (lane == 0) before = w > 0 ? P.E[round][0][1][j] : czero<R>();
        if (lane == 63) after = w < 1 ? P.E[round][1][0][j] : czero<R>();
    };
    // SO update
    publish(v, 0);
    __syncthreads();
    cx<R> u[3][L];
    {
        cx<R> vb[3], va[3];
#pragma unroll
        for (int jp = 0; jp < 3; ++jp) outer(v[jp], 0, jp, vb[jp], va[jp]);
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int t = 0; t < L; ++t) u[j][t] = v[j][t];
        if (I.sopat) so_neighbours<R, L>(u, v, vb, va, I.qa, I.qb);
#pragma unroll
        for (int t = 0; t < L; ++t)
            if (t >= len)
#pragma unroll
                for (int j = 0; j < 3; ++j) u[j][t] = czero<R>();
    }
    // right-hand side
    publish(u, 1);
    __syncthreads();
    cx<R> r[3][L];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        cx<R> ub, ua;
        outer(u[j], 1, j, ub, ua);
#pragma unroll
        for (int t = 0; t < L; ++t) {
            const cx<R> pu = t > 0 ? u[j][t > 0 ? t - 1 : 0] : ub;
            const cx<R> nu = t + 1 < L ? u[j][t + 1 < L ? t + 1 : 0] : ua;
            r[j][t] = t < len ? cn_rhs(I.rdx, u[j][t], pu + nu) : czero<R>();
        }
    }
    // elimination in 128 chunks of 4 points
    const ChunkCoef<R, L, 0> cpl(I.lx, active ? i0 : 0);
    cx<R> Ak = mk(R(1), R(0));
#pragma unroll
    for (int t = 0; t < L; ++t)
        if (t < len) Ak = Ak * (czero<R>() - cpl[t]);
    cx<R> A[3], B[3], carry[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        A[j] = Ak;
        B[j] = fwd_local<R, L>(r[j], len, cpl);
    }
    wave_scan_up3<R>(A, B, I.lv4);
    if (lane == 63)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            P.scA[0][w][j] = A[j];
            P.scB[0][w][j] = B[j];
        }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        carry[j] = w > 0 ? P.scB[0][0][j] : czero<R>();
        const cx<R> prev = shfl_up(cfma(A[j], carry[j], B[j]), 1);
        if (lane >= 1) carry[j] = prev;
    }
    fwd_fix3<R, L, 0>(r, len, cpl, carry);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        A[j] = Ak;
        B[j] = bwd_local<R, L>(r[j], len, cpl);
    }
    wave_scan_down3<R>(A, B, I.lv4);
    if (lane == 0)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            P.scA[1][w][j] = A[j];
            P.scB[1][w][j] = B[j];
        }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        carry[j] = w < 1 ? P.scB[1][1][j] : czero<R>();
        const cx<R> next = shfl_down(cfma(A[j], carry[j], B[j]), 1);
        if (lane < 63) carry[j] = next;
    }
    bwd_fix3<R, L, 0>(r, len, cpl, carry);
    // coalesced stores through this wavefront's LDS line
    cx<R> c0[L], c1[L], c2[L];
    wave_exchange<R, L>(line, lane, r[0], c0);
    wave_exchange<R, L>(line, lane, r[1], c1);
    wave_exchange<R, L>(line, lane, r[2], c2);
    if (active) {
#pragma unroll
        for (int k = 0; k < L; ++k) {
            const int i = 64 * L * w + 64 * k + lane;
            if (i < nx) {
                put2(rowp + i, c0[k]);
                put2(rowp + plane + i, c1[k]);
                put2(rowp + 2 * plane + i, c2[k]);
            }
        }
    }
    __syncthreads();  // the LDS of the pair is reused by its next row
}

template <typename R>
__device__ __forceinline__ void batch_x_item_pair(const BatchArgs<R> &a, int q, bool apply_renorm, cx<R> *line,
                                                  PairSmem<R> &P) {
    const bool active = q < a.nrows2;
    const int it = active ? a.x_items[q] : 0;
    const int inst = it >> 10, row = it & 1023;
    const BatchInst<R> &I = a.inst[active ? inst : 0];
    cx<R> *psi = a.pool + I.off;
    const double *ds = apply_renorm && active ? a.renorm + (long long)inst * 8 : nullptr;
    batch_xrow_pair<R>(I, psi, row, ds, line, P, active);
}

// x item of one wavefront (row q of the work list).
template <typename R>
__device__ __forceinline__ void batch_x_item_wave(const BatchArgs<R> &a, int q, bool apply_renorm, cx<R> *line) {
    const int it = a.x_items[q];
    const int inst = it >> 10, row = it & 1023;
    const BatchInst<R> &I = a.inst[inst];
    cx<R> *psi = a.pool + I.off;
    const double *ds = apply_renorm ? a.renorm + (long long)inst * 8 : nullptr;
    switch (I.Lx) {
    case 1: batch_xrow_wave<R, 1>(I, psi, row, ds, line); break;
    case 2: batch_xrow_wave<R, 2>(I, psi, row, ds, line); break;
    case 4: batch_xrow_wave<R, 4>(I, psi, row, ds, line); break;
    default:
        // (rows of 8-point chunks go to batch_xrow_pair where batch_pair_rows)
        if constexpr (!batch_pair_rows<R>()) batch_xrow_wave<R, 8>(I, psi, row, ds, line);
        break;
    }
}

// Elimination coefficients of a y chunk read from an LDS copy of the pivot
// head (entries from index head on equal the tail value): correct for any
// head length with no per-lane register array.
template <typename R> struct LdsCoef {
    const cx<R> *lds;
    cx<R> tail;
    int head, start;
    __device__ __forceinline__ cx<R> operator[](int t) const {
        const int i = start + t;
        return i < head ? lds[i] : tail;
    }
};

// y-line solve of one tile (TX columns x P chunks of L rows, P = 256/TX) of
// component j; returns the tile's sum of |psi|^2 (in every thread).
template <typename R, int L>
__device__ __forceinline__ double batch_ytile(const BatchInst<R> &I, cx<R> *psi, int j, int tile,
                                              BatchSmem<R> &S) {
    constexpr int TX = BatchTX<R>::v;
    constexpr int NW = BATCH_THREADS / 64;
    const int nx = I.nx, ny = I.ny;
    const long long plane = (long long)nx * ny;
    const int tid = threadIdx.x, c = tid % TX, k = tid / TX;
    const int lane = tid & 63, wave = tid >> 6;
    const int x = tile * TX + c;
    const bool valid = x < nx;
    const int start = k * L;
    const int len = valid ? max(0, min(L, ny - start)) : 0;
    cx<R> *col = psi + j * plane + (valid ? x : 0);
    const int head = min(I.ly.head, ny);
    for (int i = tid; i < head; i += BATCH_THREADS) S.line[i] = I.ly.cp[i];
    cx<R> f[L];
#pragma unroll
    for (int t = 0; t < L; ++t) f[t] = t < len ? col[(long long)(start + t) * nx] : czero<R>();
    const cx<R> fl = (len > 0 && start >= 1) ? col[(long long)(start - 1) * nx] : czero<R>();
    const cx<R> fr = (len > 0 && start + len < ny) ? col[(long long)(start + len) * nx] : czero<R>();
    cx<R> r[L];
#pragma unroll
    for (int t = 0; t < L; ++t) {
        if (t < len) {
            const cx<R> left = t == 0 ? fl : f[t > 0 ? t - 1 : 0];
            const cx<R> right = (t + 1 < L && t + 1 < len) ? f[t + 1 < L ? t + 1 : 0] : fr;
            r[t] = cn_rhs(I.rdy, f[t], left + right);
        } else {
            r[t] = czero<R>();
        }
    }
    const LdsCoef<R> cpl{S.line, I.ly.cp_inf, head, start};
    const cx<R> Ak = I.ly.chunkA[k];
    __syncthreads();  // the pivot head is staged
    cx<R> A = Ak;
    cx<R> Bv = fwd_local<R, L>(r, len, cpl);
    wave_scan_up<R, TX>(A, Bv, I.ly.levels);
    if (lane >= 64 - TX) {
        S.scA[0][wave][c] = A;
        S.scB[0][wave][c] = Bv;
    }
    __syncthreads();
    cx<R> carry = czero<R>();
    for (int w = 0; w < wave; ++w) carry = cfma(S.scA[0][w][c], carry, S.scB[0][w][c]);
    {
        const cx<R> incl = cfma(A, carry, Bv);
        const cx<R> prev = shfl_up(incl, TX);
        if (lane >= TX) carry = prev;
    }
    fwd_fix<R, L>(r, len, cpl, carry);
    asm volatile("" ::: "memory");  // re-read the coefficients rather than keep L of them live
    A = Ak;
    Bv = bwd_local<R, L>(r, len, cpl);
    wave_scan_down<R, TX>(A, Bv, I.ly.levels);
    if (lane < TX) {
        S.scA[1][wave][c] = A;
        S.scB[1][wave][c] = Bv;
    }
    __syncthreads();
    carry = czero<R>();
    for (int w = NW - 1; w > wave; --w) carry = cfma(S.scA[1][w][c], carry, S.scB[1][w][c]);
    {
        const cx<R> incl = cfma(A, carry, Bv);
        const cx<R> next = shfl_down(incl, TX);
        if (lane < 64 - TX) carry = next;
    }
    bwd_fix<R, L>(r, len, cpl, carry);
    double nrm = 0.0;
#pragma unroll
    for (int t = 0; t < L; ++t) {
        if (t < len) {
            col[(long long)(start + t) * nx] = r[t];
            nrm += (double)abs2(r[t]);
        }
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) nrm += __shfl_down(nrm, d, 64);
    if (lane == 0) S.red[0][wave] = nrm;
    __syncthreads();
    double tot = 0.0;
    for (int w = 0; w < NW; ++w) tot += S.red[0][w];
    __syncthreads();
    return tot;
}

// R item: fixed-order sums of an instance's tile partials and its RENORM
// factors.
template <typename R> __device__ __forceinline__ void batch_renorm_item(const BatchArgs<R> &a, int inst,
                                                                        BatchSmem<R> &S) {
    const BatchInst<R> &I = a.inst[inst];
    const int t = threadIdx.x;
    for (int j = 0; j < 3; ++j) {
        double s = 0.0;
        for (int q = t; q < I.ntiles; q += BATCH_THREADS) s += a.partials[(long long)(I.tile_base + q) * 3 + j];
        S.red[j][t] = s;
    }
    __syncthreads();
    for (int w = BATCH_THREADS / 2; w >= 1; w >>= 1) {
        if (t < w)
            for (int j = 0; j < 3; ++j) S.red[j][t] += S.red[j][t + w];
        __syncthreads();
    }
    if (t == 0) {
        double N[3] = {S.red[0][0] * I.sp.dA, S.red[1][0] * I.sp.dA, S.red[2][0] * I.sp.dA};
        double d[3], fb = 0.0;
        renorm_factors(I.sp, N, d, &fb);
        double *o = a.renorm + (long long)inst * 8;
        for (int j = 0; j < 3; ++j) {
            o[j] = d[j];
            o[3 + j] = N[j];
        }
        o[6] = fb;
    }
    __syncthreads();
}

// ------------------------------------------------------------- items ---
template <typename R>
__device__ __forceinline__ void batch_y_item(const BatchArgs<R> &a, int q, BatchSmem<R> &S) {
    const int it = a.y_items[q];
    const int inst = it >> 8, j = (it >> 6) & 3, tile = it & 63;
    const BatchInst<R> &I = a.inst[inst];
    cx<R> *psi = a.pool + I.off;
    double s;
    switch (I.Ly) {
    case 1: s = batch_ytile<R, 1>(I, psi, j, tile, S); break;
    case 2: s = batch_ytile<R, 2>(I, psi, j, tile, S); break;
    case 4: s = batch_ytile<R, 4>(I, psi, j, tile, S); break;
    case 8: s = batch_ytile<R, 8>(I, psi, j, tile, S); break;
    case 16: s = batch_ytile<R, 16>(I, psi, j, tile, S); break;
    default: s = batch_ytile<R, (BatchTX<R>::v == 8 ? 16 : 32)>(I, psi, j, tile, S); break;
    }
    if (threadIdx.x == 0) a.partials[(long long)(I.tile_base + tile) * 3 + j] = s;
}

template <typename R> __device__ __forceinline__ void batch_scale_item(const BatchArgs<R> &a, int q) {
    const int it = a.x_items[q];
    const int inst = it >> 10, row = it & 1023;
    const BatchInst<R> &I = a.inst[inst];
    const double *dd = a.renorm + (long long)inst * 8;
    const R d[3] = {R(coherent_load(dd)), R(coherent_load(dd + 1)), R(coherent_load(dd + 2))};
    cx<R> *rowp = a.pool + I.off + (long long)row * I.nx;
    const long long plane = (long long)I.nx * I.ny;
    for (int i = threadIdx.x; i < I.nx; i += BATCH_THREADS)
#pragma unroll
        for (int j = 0; j < 3; ++j) rowp[j * plane + i] = d[j] * rowp[j * plane + i];
}

// ----------------------------------------------------------- kernels ---
// Persistent: every workgroup resident, items assigned round-robin.
template <typename R>
__global__ void __launch_bounds__(BATCH_THREADS) batch_persistent_kernel(BatchArgs<R> a) {
    __shared__ BatchSmem<R> S;
    __shared__ cx<R> xlines[BATCH_THREADS / 64][bx_line_slots<R, BATCH_MAX_LX>()];
    __shared__ PairSmem<R> pairs[BATCH_THREADS / 128];
    const int wave = threadIdx.x >> 6, pair = threadIdx.x >> 7;
    for (int step = 0; step < a.nsteps; ++step) {
        // x rows by two wavefronts (every pair runs the same number of rounds)
        for (int q0 = blockIdx.x * (BATCH_THREADS / 128); q0 < a.nrows2; q0 += gridDim.x * (BATCH_THREADS / 128))
            batch_x_item_pair(a, q0 + pair, step > 0, xlines[wave], pairs[pair]);
        // the other x rows, one per wavefront
        for (int q = a.nrows2 + blockIdx.x * (BATCH_THREADS / 64) + wave; q < a.nrows;
             q += gridDim.x * (BATCH_THREADS / 64))
            batch_x_item_wave(a, q, step > 0, xlines[wave]);
        if (!grid_sync(a.bar, a.spin_limit)) return;
        for (int q = blockIdx.x; q < a.nyitems; q += gridDim.x) batch_y_item(a, q, S);
        if (!grid_sync(a.bar, a.spin_limit)) return;
        for (int q = blockIdx.x; q < a.ninst; q += gridDim.x) batch_renorm_item(a, q, S);
        if (!grid_sync(a.bar, a.spin_limit)) return;
    }
    if (a.nsteps > 0)
        for (int q = blockIdx.x; q < a.nrows; q += gridDim.x) batch_scale_item(a, q);
}

// One launch per phase: one workgroup per item (x rows: one wavefront per
// row, BATCH_XWAVES rows per workgroup).
constexpr int BATCH_XWAVES = 4;
template <typename R>
__global__ void __launch_bounds__(64 * BATCH_XWAVES) batch_x_kernel(BatchArgs<R> a, int apply_renorm) {
    __shared__ cx<R> xlines[BATCH_XWAVES][bx_line_slots<R, BATCH_MAX_LX>()];
    const int wave = threadIdx.x >> 6;
    const int q = a.nrows2 + blockIdx.x * BATCH_XWAVES + wave;
    if (q < a.nrows) batch_x_item_wave(a, q, apply_renorm != 0, xlines[wave]);
}

// The rows by two wavefronts: one row per workgroup of 128 threads.
template <typename R>
__global__ void __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(4))) batch_x2_kernel(BatchArgs<R> a, int apply_renorm) {
    __shared__ cx<R> xlines[2][bx_line_slots<R, 4>()];
    __shared__ PairSmem<R> P;
    batch_x_item_pair(a, blockIdx.x, apply_renorm != 0, xlines[threadIdx.x >> 6], P);
}

template <typename R>
__global__ void __launch_bounds__(BATCH_THREADS) batch_y_kernel(BatchArgs<R> a) {
    __shared__ BatchSmem<R> S;
    batch_y_item(a, blockIdx.x, S);
}

template <typename R>
__global__ void __launch_bounds__(BATCH_THREADS) batch_renorm_kernel(BatchArgs<R> a) {
    __shared__ BatchSmem<R> S;
    batch_renorm_item(a, a.r_items ? a.r_items[blockIdx.x] : (int)blockIdx.x, S);
}

template <typename R>
__global__ void __launch_bounds__(BATCH_THREADS) batch_scale_kernel(BatchArgs<R> a) {
    batch_scale_item(a, blockIdx.x);
}

} // namespace ssgp
