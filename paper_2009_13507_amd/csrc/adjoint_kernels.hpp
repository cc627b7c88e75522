// adjoint_kernels.hpp -- reverse-mode derivative of one real-time SS-CN step.
//
// Gradient convention: g = dL/dRe(psi) + i dL/dIm(psi), so that for a linear
// map M the pull-back is M^H g.  A step is CNy o CNx o SO o HERM o CALCNU;
// its adjoint runs in reverse:
//   CN^H:   for M = (I + sT)^-1 (I - sT) with T real symmetric,
//           M^H = (I + s*T)^-1 (I - s*T): the y-pass / x-line solve with the
//           conjugate factor (s = i dt/2 -> -i dt/2);
//   SO^H:   S = I - i dt H with H Hermitian, so S^H = I + i dt H;
//   HERM^T: y = U(A(psi)) psi with U = I + f(w) A + h(w) A^2, w = |a|^2+|b|^2
//           (see step_kernels.hpp).  For a real loss
//             <g, dy>_R = <U^H g, dpsi>_R + Re(da Qa) + Re(db Qb),
//           where, with the pairs (u, v) in {(f* g, psi), (h A g, psi),
//           (h g, A psi)} and kw = Re(f' g^H A psi + h' g^H A^2 psi),
//             Qa = sum (u_{+1}^* v_0 + u_0 v_{+1}^*) + 2 kw a^*,
//             Qb = sum (u_0^* v_{-1} + u_{-1} v_0^*) + 2 kw b^*,
//           and da, db follow from a = c2 psi_{-1}^* psi_0 + Omega~,
//           b = c2 psi_0^* psi_{+1} + Omega~; the Omega derivative of the
//           loss is Re(Qa + Qb)/sqrt(2);
//   CALCNU^T: y_j = e_j psi_j, e_j = exp(-i dt phi_j(rho)) with
//           Phi_jm = dphi_j/drho_m:  g_m <- e_m^* g_m
//             + 2 dt psi_m sum_j Phi_jm Im(g_j^* y_j).
// The x-pass of the adjoint reads lambda and the step input psi^n and writes
// lambda: the pointwise forward values are recomputed, not stored.
#pragma once
#include "step_kernels.hpp"

namespace ssgp {

// dS/dq for S(q) = sin(u)/u, q = u^2:
//   series sum_k (k+1) (-1)^(k+1) q^k / (2k+3)!, closed form (cos u - S)/(2q).
template <typename R> __device__ __forceinline__ R dsinc_q(R q) {
    if (q <= SeriesLimit<R>::q) {
        R acc = R(0);
#pragma unroll
        for (int k = 9; k >= 0; --k) {
            const R c = R((k + 1) * inv_fact(2 * k + 3));
            acc = fma_(-q, acc, -c);
        }
        // acc = sum_k (-1)^(k+1) (k+1) q^k/(2k+3)! built as -c0 - q(-c1 - q(...))
        return acc;
    }
    const R u = sqrt_(q);
    R su, cu;
    sincos_(u, &su, &cu);
    return (cu - su / u) / (R(2) * q);
}

template <typename R>
__device__ __forceinline__ void Amul(cx<R> a, cx<R> b, const cx<R> v[3], cx<R> o[3]) {
    o[0] = a * v[1];
    o[1] = cfma(conj(a), v[0], b * v[2]);
    o[2] = conj(b) * v[1];
}

// g: in the gradient w.r.t. the HERM output, out the gradient w.r.t. the
// step input psi.  Returns the Omega derivative at this point.
template <typename R>
__device__ __forceinline__ R pointwise_adjoint_real(const cx<R> psi[3], cx<R> g[3], R V, const Model<R> &M) {
    const R dt = M.dt;
    R rj[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) rj[j] = abs2(psi[j]);
    const R rho = rj[0] + rj[1] + rj[2];
    const R base = V + M.c0 * rho;
    const R phi[3] = {base + M.c2 * (rj[0] - rj[2] + rj[1]), base + M.c2 * (rj[0] + rj[2]),
                      base + M.c2 * (rj[2] - rj[0] + rj[1])};
    cx<R> e[3], y[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        R c, s;
        cos_sin(dt * phi[j], c, s);
        e[j] = mk(c, -s);
        y[j] = psi[j] * e[j];
    }
    // HERM at y
    const cx<R> a = cfma(mk(M.c2, R(0)), conj(y[2]) * y[1], mk(M.om_t, R(0)));
    const cx<R> b = cfma(mk(M.c2, R(0)), conj(y[1]) * y[0], mk(M.om_t, R(0)));
    const R q = R(0.25) * dt * dt * (abs2(a) + abs2(b));
    R S, C;
    if (q <= SeriesLimit<R>::q) {
        S = sinc_q(q);
        C = cos_q(q);
    } else {
        const R u = sqrt_(q);
        R su, cu;
        sincos_(u, &su, &cu);
        S = su / u;
        C = cu;
    }
    const R Sp = dsinc_q(q);
    // f = i fi, h real; f' = i fpi, h' = hp (derivatives with respect to w)
    const R fi = -dt * S * C;
    const R h = R(-0.5) * dt * dt * S * S;
    const R fpi = -dt * (Sp * C - R(0.5) * S * S) * R(0.25) * dt * dt;
    const R hp = R(-0.25) * dt * dt * dt * dt * S * Sp;
    cx<R> Av[3], A2v[3], Ag[3], A2g[3];
    Amul(a, b, y, Av);
    Amul(a, b, Av, A2v);
    Amul(a, b, g, Ag);
    Amul(a, b, Ag, A2g);
    cx<R> gAv = czero<R>(), gA2v = czero<R>();
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        gAv = cfma(conj(g[j]), Av[j], gAv);
        gA2v = cfma(conj(g[j]), A2v[j], gA2v);
    }
    const R kw = -fpi * gAv.y + hp * gA2v.x;
    // pairs (u, v): (f^* g, y), (h A g, y), (h g, A y); f^* = -i fi
    cx<R> u1[3], u2[3], u3[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        u1[j] = (-fi) * mul_i(g[j]);
        u2[j] = h * Ag[j];
        u3[j] = h * g[j];
    }
    cx<R> Pa = czero<R>(), Pb = czero<R>();
    const cx<R> *us[3] = {u1, u2, u3};
    const cx<R> *vs[3] = {y, y, Av};
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        const cx<R> *u = us[t], *v = vs[t];
        Pa = Pa + conj(u[0]) * v[1] + u[1] * conj(v[0]);
        Pb = Pb + conj(u[1]) * v[2] + u[2] * conj(v[1]);
    }
    const cx<R> Qa = Pa + (R(2) * kw) * conj(a);
    const cx<R> Qb = Pb + (R(2) * kw) * conj(b);
    // U^H g = g + f^* A g + h A^2 g, plus the terms through a and b
    cx<R> ga[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) ga[j] = g[j] + (-fi) * mul_i(Ag[j]) + h * A2g[j];
    ga[0] = ga[0] + M.c2 * (y[1] * conj(Qb));
    ga[1] = ga[1] + M.c2 * (y[2] * conj(Qa) + y[0] * Qb);
    ga[2] = ga[2] + M.c2 * (y[1] * Qa);
    // CALCNU^T
    R t[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) t[j] = (conj(ga[j]) * y[j]).y;
    const R cpp = M.c0 + M.c2, cpm = M.c0 - M.c2;
    // c_m = sum_j Phi_jm t_j with Phi = [[c0+c2, c0+c2, c0-c2], [c0+c2, c0, c0+c2], [c0-c2, c0+c2, c0+c2]]
    const R cm[3] = {cpp * t[0] + cpp * t[1] + cpm * t[2], cpp * t[0] + M.c0 * t[1] + cpp * t[2],
                     cpm * t[0] + cpp * t[1] + cpp * t[2]};
#pragma unroll
    for (int j = 0; j < 3; ++j) g[j] = conj(e[j]) * ga[j] + (R(2) * dt * cm[j]) * psi[j];
    return (Qa.x + Qb.x) * R(0.70710678118654752440);
}

template <typename R> struct AdjXArgs {
    cx<R> *lam;                // gradient, updated in place (one row per workgroup)
    const cx<R> *psi_n;        // step input
    int nx, ny;
    long long plane;
    R dx, dy, x0, y0;
    Model<R> m;
    LineCoef<R> cx_;           // CN_x coefficients with the conjugate factor
    cx<R> rdiag;               // diagonal of (I - sT)/o (off-diagonal -1)
    cx<R> qx[9];               // SO^H stencil couplings
    unsigned qxmask;
    int sopat;                 // what the kernel reads of qx (set by its launcher, so_pattern):
    cx<R> qa, qb;              // 1 neighbouring components, 2 diagonal, 0 none
    double *omega_partials;    // [ny] per-row Omega derivative
};

// One row per workgroup of 4 wavefronts: wavefronts 0-2 solve the three
// CN_x^H lines, all four share the pointwise part (SO^H and the transposed
// HERM/CALCNU, the bulk of the arithmetic, about 206 VGPRs: 2 wavefronts per
// SIMD).  Measured faster than 3, 6 or 8 wavefronts per row.
constexpr int ADJ_THREADS = 256;

template <typename R, int L, int CM>
__global__ void __launch_bounds__(ADJ_THREADS) adj_xpass_kernel(AdjXArgs<R> a) {
    extern __shared__ unsigned char smem_raw[];
    cx<R> *s = reinterpret_cast<cx<R> *>(smem_raw);
    __shared__ double red[ADJ_THREADS / 64];
    const int nx = a.nx;
    const int ld = srow<L>(nx);
    const int row = blockIdx.x;
    const int tid = threadIdx.x;
    const long long roff = (long long)row * nx;
    cx<R> *lam = a.lam + roff;
    const cx<R> *psi = a.psi_n + roff;

    for (int i = tid; i < nx; i += ADJ_THREADS) {
        const int si = sidx<L>(i);
        s[si] = lam[i];
        s[ld + si] = lam[a.plane + i];
        s[2 * ld + si] = lam[2 * a.plane + i];
    }
    __syncthreads();
    // CN_x^H per component
    if (tid < 192) {
        const int j = tid >> 6, lane = tid & 63;
        const int start = lane * L;
        const int len = max(0, min(L, nx - start));
        cx<R> *sj = s + j * ld;
        auto at = [&](int i) -> cx<R> { return (i < 0 || i >= nx) ? czero<R>() : sj[sidx<L>(i)]; };
        cx<R> r[L];
        cx<R> um = czero<R>(), uc = czero<R>();
        if (len > 0) {
            um = at(start - 1);
            uc = at(start);
        }
#pragma unroll
        for (int t = 0; t < L; ++t) {
            if (t < len) {
                const cx<R> un = at(start + t + 1);
                r[t] = cn_rhs(a.rdiag, uc, um + un);
                um = uc;
                uc = un;
            } else {
                r[t] = czero<R>();
            }
        }
        solve_line_wave<R, L, CM>(r, start, len, a.cx_);
#pragma unroll
        for (int t = 0; t < L; ++t)
            if (t < len) sj[sidx<L>(start + t)] = r[t];
    }
    __syncthreads();
    // SO^H stencil, then the pointwise transpose, in the coalesced layout
    const R yv = a.y0 + R(row) * a.dy;
    const R vy = R(0.5) * a.m.kappa2 * yv * yv;
    double dom = 0.0;
    for (int i = tid; i < nx; i += ADJ_THREADS) {
        cx<R> g[3], p[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            g[j] = s[j * ld + sidx<L>(i)];
            p[j] = psi[j * a.plane + i];
        }
        // SO^H: the terms of each component in the order j' = 0, 1, 2
        auto diff = [&](int jp) {
            const cx<R> fp = i + 1 < nx ? s[jp * ld + sidx<L>(i + 1)] : czero<R>();
            const cx<R> fm = i >= 1 ? s[jp * ld + sidx<L>(i - 1)] : czero<R>();
            return fp - fm;
        };
        if (a.sopat == 1) {
            const cx<R> d0 = diff(0), d1 = diff(1), d2 = diff(2);
            g[0] = cfma(a.qa, d1, g[0]);
            g[1] = cfma(a.qa, d2, cfma(a.qb, d0, g[1]));
            g[2] = cfma(a.qb, d1, g[2]);
        } else if (a.sopat == 2) {
            g[0] = cfma(a.qa, diff(0), g[0]);
            g[2] = cfma(a.qb, diff(2), g[2]);
        }
        const R xv = a.x0 + R(i) * a.dx;
        dom += (double)pointwise_adjoint_real(p, g, R(0.5) * xv * xv + vy, a.m);
#pragma unroll
        for (int j = 0; j < 3; ++j) lam[j * a.plane + i] = g[j];
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) dom += __shfl_down(dom, d, 64);
    if ((tid & 63) == 0) red[tid >> 6] = dom;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int w = 0; w < ADJ_THREADS / 64; ++w) t += red[w];
        a.omega_partials[row] = t;
    }
}

} // namespace ssgp
