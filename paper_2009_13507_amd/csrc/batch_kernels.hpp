// batch_kernels.hpp -- many independent 2D grids (uneven sizes and
// parameters) advanced together in imaginary time.
//
// Per step, over all instances of the batch:
//   X phase, items (instance, row): RENORM scale of the previous step,
//      CALCNU, HERM, SO, the Crank-Nicolson right-hand side and the x-line
//      solve of one row (one item per 4-wavefront workgroup: the pointwise
//      part in a coalesced layout, then each component line transposed
//      through LDS into 64 chunks and solved by one wavefront; for rows of at
//      most 512 points this measured faster than the single-grid row code);
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
// a generation word (vector atomics at agent scope, with fences on both
// sides so that the state written before the barrier is visible after it on
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
    cx<R> rdx, rdy;            // diagonal of (I - sT)/o of x and y (off-diagonal -1)
    cx<R> qx[9];               // SO: psi'_j += sum_j' qx[j][j'] (psi_j'(i+1) - psi_j'(i-1))
    unsigned qxmask;
    RenormSpec sp;
};

template <typename R> struct BatchArgs {
    cx<R> *pool;
    const BatchInst<R> *inst;
    const int *x_items;        // (instance << 10) | row
    const int *y_items;        // (instance << 8) | (component << 6) | tile
    int nrows, nyitems;
    double *partials;          // [total tiles][3] tile sums of |psi|^2
    double *renorm;            // [instances][8]: d[3], N[3], fallback
    int ninst;
    unsigned *bar;             // [0] arrivals, [1] generation, [2] stop, [3] sticky timeout flag
    int nsteps;
    long long spin_limit;
};

__device__ __forceinline__ double coherent_load(const double *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Device-wide barrier; returns false when the grid must stop.
__device__ __forceinline__ bool grid_sync(unsigned *bar, long long spin_limit) {
    __shared__ int stop;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned gen = __hip_atomic_load(bar + 1, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned arrived = __hip_atomic_fetch_add(bar, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (arrived == gridDim.x - 1) {
            __hip_atomic_store(bar, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(bar + 1, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            long long spins = 0;
            while (__hip_atomic_load(bar + 1, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                if (__hip_atomic_load(bar + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) break;
                if (++spins > spin_limit) {
                    __hip_atomic_store(bar + 2, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        stop = __hip_atomic_load(bar + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
    }
    __syncthreads();
    __threadfence();
    return !stop;
}

// Shared memory of one workgroup.
template <typename R> struct BatchSmem {
    cx<R> line[64 * BATCH_MAX_LX + 64 + 1];  // one staged row, one padding slot per chunk
    cx<R> edge[48];                          // x edge exchange: [2][4 waves][2 ends][3 comps]
    cx<R> scA[2][4][BatchTX<R>::v], scB[2][4][BatchTX<R>::v];
    double red[3][BATCH_THREADS];
};

// One x row of one instance (the single-grid x-pass algorithm, 4 waves).
template <typename R, int L>
__device__ __forceinline__ void batch_xrow(const BatchInst<R> &I, cx<R> *psi, int row, const double *dscale,
                                           BatchSmem<R> &S) {
    constexpr int KM = (64 * L + BATCH_THREADS - 1) / BATCH_THREADS;
    cx<R> *B = S.line;
    cx<R> *E = S.edge;
    const int nx = I.nx;
    const long long plane = (long long)nx * I.ny;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int K = (nx + BATCH_THREADS - 1) / BATCH_THREADS;
    const int RW = 64 * K;
    cx<R> *rowp = psi + (long long)row * nx;
    cx<R> v[3][KM];
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        const int i = w * RW + 64 * k + lane;
        const bool ok = k < K && i < nx;
#pragma unroll
        for (int j = 0; j < 3; ++j) v[j][k] = ok ? rowp[j * plane + i] : czero<R>();
    }
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
        for (int k = 0; k < KM; ++k) {
            const int i = w * RW + 64 * k + lane;
            if (k < K && i < nx) {
                if (dscale) {
                    v[0][k] = d0 * v[0][k];
                    v[1][k] = d1 * v[1][k];
                    v[2][k] = d2 * v[2][k];
                }
                const R xv = I.x0 + R(i) * I.dx;
                pointwise(v[0][k], v[1][k], v[2][k], R(0.5) * xv * xv + vy, I.m);
            }
        }
    }
    auto exchange_edges = [&](cx<R> (&x)[3][KM], int round) {
        cx<R> *Er = E + round * 24;
#pragma unroll
        for (int k = 0; k < KM; ++k)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                if (lane == 0 && k == 0) Er[(w * 2 + 0) * 3 + j] = x[j][k];
                if (lane == 63 && k == K - 1) Er[(w * 2 + 1) * 3 + j] = x[j][k];
            }
    };
    auto neighbours = [&](cx<R> (&x)[3][KM], int round, int j, int k, cx<R> &prev, cx<R> &next) {
        const cx<R> *Er = E + round * 24;
        const cx<R> r0 = ror1(x[j][k]);
        const cx<R> rm = ror1(x[j][k > 0 ? k - 1 : 0]);
        const cx<R> l0 = rol1(x[j][k]);
        const cx<R> lp = rol1(x[j][k + 1 < KM ? k + 1 : k]);
        prev = r0;
        next = l0;
        if (lane == 0) prev = k > 0 ? rm : (w > 0 ? Er[((w - 1) * 2 + 1) * 3 + j] : czero<R>());
        if (lane == 63) next = k < K - 1 ? lp : (w < 3 ? Er[((w + 1) * 2 + 0) * 3 + j] : czero<R>());
    };
    // SO update
    exchange_edges(v, 0);
    __syncthreads();
    cx<R> u[3][KM];
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        cx<R> pv[3], nv[3];
#pragma unroll
        for (int jp = 0; jp < 3; ++jp) neighbours(v, 0, jp, k, pv[jp], nv[jp]);
        const int i = w * RW + 64 * k + lane;
        const bool ok = k < K && i < nx;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cx<R> t = v[j][k];
#pragma unroll
            for (int jp = 0; jp < 3; ++jp)
                if (I.qxmask & (1u << (3 * j + jp))) t = cfma(I.qx[3 * j + jp], nv[jp] - pv[jp], t);
            u[j][k] = ok ? t : czero<R>();
        }
    }
    // right-hand side (I - sT) u / o
    exchange_edges(u, 1);
    __syncthreads();
    cx<R> r[3][KM];
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        const int i = w * RW + 64 * k + lane;
        const bool ok = k < K && i < nx;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cx<R> pu, nu;
            neighbours(u, 1, j, k, pu, nu);
            r[j][k] = ok ? cn_rhs(I.rdx, u[j][k], pu + nu) : czero<R>();
        }
    }
    // transpose into the chunk layout, solve (waves 0-2), transpose back
    const int start = lane * L;
    const int len = max(0, min(L, nx - start));
    cx<R> c[L];
#pragma unroll
    for (int jj = 0; jj < 3; ++jj) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < KM; ++k) {
            const int i = w * RW + 64 * k + lane;
            if (k < K && i < nx) B[sidx<L>(i)] = r[jj][k];
        }
        __syncthreads();
        if (w == jj) {
#pragma unroll
            for (int t = 0; t < L; ++t) c[t] = t < len ? B[sidx<L>(start + t)] : czero<R>();
        }
    }
    if (w < 3) solve_line_wave<R, L, 0>(c, start, len, I.lx);
#pragma unroll
    for (int jj = 0; jj < 3; ++jj) {
        __syncthreads();
        if (w == jj) {
#pragma unroll
            for (int t = 0; t < L; ++t)
                if (t < len) B[sidx<L>(start + t)] = c[t];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < KM; ++k) {
            const int i = w * RW + 64 * k + lane;
            if (k < K && i < nx) rowp[jj * plane + i] = B[sidx<L>(i)];
        }
    }
    __syncthreads();  // the shared buffers are reused by the next item
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
__device__ __forceinline__ void batch_x_item(const BatchArgs<R> &a, int q, bool apply_renorm, BatchSmem<R> &S) {
    const int it = a.x_items[q];
    const int inst = it >> 10, row = it & 1023;
    const BatchInst<R> &I = a.inst[inst];
    cx<R> *psi = a.pool + I.off;
    const double *ds = apply_renorm ? a.renorm + (long long)inst * 8 : nullptr;
    switch (I.Lx) {
    case 1: batch_xrow<R, 1>(I, psi, row, ds, S); break;
    case 2: batch_xrow<R, 2>(I, psi, row, ds, S); break;
    case 4: batch_xrow<R, 4>(I, psi, row, ds, S); break;
    default: batch_xrow<R, 8>(I, psi, row, ds, S); break;
    }
}

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
    for (int step = 0; step < a.nsteps; ++step) {
        for (int q = blockIdx.x; q < a.nrows; q += gridDim.x) batch_x_item(a, q, step > 0, S);
        if (!grid_sync(a.bar, a.spin_limit)) return;
        for (int q = blockIdx.x; q < a.nyitems; q += gridDim.x) batch_y_item(a, q, S);
        if (!grid_sync(a.bar, a.spin_limit)) return;
        for (int q = blockIdx.x; q < a.ninst; q += gridDim.x) batch_renorm_item(a, q, S);
        if (!grid_sync(a.bar, a.spin_limit)) return;
    }
    if (a.nsteps > 0)
        for (int q = blockIdx.x; q < a.nrows; q += gridDim.x) batch_scale_item(a, q);
}

// One launch per phase: one workgroup per item.
template <typename R>
__global__ void __launch_bounds__(BATCH_THREADS) batch_x_kernel(BatchArgs<R> a, int apply_renorm) {
    __shared__ BatchSmem<R> S;
    batch_x_item(a, blockIdx.x, apply_renorm != 0, S);
}

template <typename R>
__global__ void __launch_bounds__(BATCH_THREADS) batch_y_kernel(BatchArgs<R> a) {
    __shared__ BatchSmem<R> S;
    batch_y_item(a, blockIdx.x, S);
}

template <typename R>
__global__ void __launch_bounds__(BATCH_THREADS) batch_renorm_kernel(BatchArgs<R> a) {
    __shared__ BatchSmem<R> S;
    batch_renorm_item(a, blockIdx.x, S);
}

template <typename R>
__global__ void __launch_bounds__(BATCH_THREADS) batch_scale_kernel(BatchArgs<R> a) {
    batch_scale_item(a, blockIdx.x);
}

} // namespace ssgp
