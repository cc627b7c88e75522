// step_kernels.hpp -- the SS-CN time step on gfx950.
//
// One step of the spin-1 GP equations (Sec. 3 and App. A of the paper) is
// two device-wide passes over the state:
//   x-pass (one workgroup of 4 wavefronts per row, KM consecutive points per
//          thread): the RENORM of the previous imaginary-time step, CALCNU,
//          HERM, the SO update and the Crank-Nicolson right-hand side, and
//          the chunked elimination of the three x lines in the same layout;
//          coalesced stores through a per-wavefront LDS line;
//   y-pass (one workgroup per tile of 4 columns and one component): the
//          Crank-Nicolson solve along y, column chunks held in registers, plus
//          the per-tile sums of |psi|^2 for the imaginary-time RENORM.
// The 1D kernel keeps a whole 1D run in one workgroup's LDS.
//
// Chunked Thomas elimination.  The matrix I + sT of every line is the same
// Toeplitz tridiagonal, so the pivots are line independent and tabulated on
// the host: with c'_i = o / m_i (o the off-diagonal, m_i the pivots) the
// forward sweep is y_i = c'_i (r_i/o - y_{i-1}) and the back substitution
// x_i = y_i - c'_i x_{i+1}.  Each lane owns a contiguous chunk of points.
// Both sweeps are first-order linear recurrences with the multiplier -c'_i,
// so a lane first runs its chunk with zero carry-in, the chunks are joined by
// a scan of the affine maps Y_k = A_k Y_{k-1} + B_k (A_k = prod over the
// chunk of -c'_i, tabulated), and each lane adds the carried term.  The scan
// depth within a wavefront drops carries from chunks so far back that their
// weight is below 2^-64 (LineCoef::levels); the result is Thomas elimination
// up to rounding order.
#pragma once
#include "cplx.hpp"

namespace ssgp {

template <typename R> struct Model {
    R c0, c2, dt, om_t, kappa2;  // om_t = Omega / sqrt(2)
    int imag;                    // 1: imaginary time (k = 1), 0: real time (k = i)
};

// --------------------------------------------------------------- math ---
__device__ __forceinline__ void sincos_(double x, double *s, double *c) { sincos(x, s, c); }
__device__ __forceinline__ void sincos_(float x, float *s, float *c) { sincosf(x, s, c); }
__device__ __forceinline__ double exp_(double x) { return exp(x); }
__device__ __forceinline__ float exp_(float x) { return expf(x); }
__device__ __forceinline__ double sinh_(double x) { return sinh(x); }
__device__ __forceinline__ float sinh_(float x) { return sinhf(x); }
__device__ __forceinline__ double cosh_(double x) { return cosh(x); }
__device__ __forceinline__ float cosh_(float x) { return coshf(x); }
__device__ __forceinline__ double sqrt_(double x) { return sqrt(x); }
__device__ __forceinline__ float sqrt_(float x) { return sqrtf(x); }

// cos(th), sin(th); Taylor series for |th| <= pi/4 (as short as every lane
// of the wavefront allows), library call beyond.
template <typename R, int N> __device__ __forceinline__ void cos_sin_n(R th, R q, R &c, R &s) {
    s = th * series_q<R, true, 1, N>(q);
    c = series_q<R, true, 0, N>(q);
}
template <typename R> __device__ __forceinline__ void cos_sin(R th, R &c, R &s) {
    const R q = th * th;
    if (__all(q <= R(SERIES_Q4))) {
        cos_sin_n<R, 4>(th, q, c, s);
    } else if (__all(q <= R(SERIES_Q5))) {
        cos_sin_n<R, 5>(th, q, c, s);
    } else if (__all(q <= R(SERIES_Q6))) {
        cos_sin_n<R, 6>(th, q, c, s);
    } else if (q <= SeriesLimit<R>::q) {
        s = th * sinc_q(q);
        c = cos_q(q);
    } else {
        sincos_(th, &s, &c);
    }
}

// CALCNU then HERM at one grid point (V = trap potential there).
//  CALCNU: psi_j <- exp(-k dt phi_j) psi_j, the three phi_j from the input
//          densities (square brackets of Eqs. (1)-(2)).
//  HERM:   psi <- exp(-k dt A) psi, A of App. A Eq. (eq:nu).  With
//          C^2 = |a|^2 + |b|^2 the eigenvalues are C, 0, -C, so A^3 = C^2 A and
//            exp(-i dt A) = I - i (sin(C dt)/C) A + ((cos(C dt) - 1)/C^2) A^2,
//            exp(-dt A)   = I - (sinh(C dt)/C) A + ((cosh(C dt) - 1)/C^2) A^2.
//          With u = C dt / 2: sin(C dt)/C = dt sinc(u) cos(u) and
//          (cos(C dt) - 1)/C^2 = -(dt^2/2) sinc(u)^2 (hyperbolic analogues in
//          imaginary time), all series in u^2 = dt^2 C^2 / 4: no square
//          root, no division, and no special case at C = 0.

// The three CALCNU exponents dt phi_j at one point.
template <typename R>
__device__ __forceinline__ void calcnu_phases(const cx<R> &p, const cx<R> &z, const cx<R> &m, R V,
                                              const Model<R> &M, R (&th)[3]) {
    const R rp = abs2(p), r0 = abs2(z), rm = abs2(m);
    const R base = V + M.c0 * (rp + r0 + rm);
    th[0] = M.dt * (base + M.c2 * (rp - rm + r0));
    th[1] = M.dt * (base + M.c2 * (rp + rm));
    th[2] = M.dt * (base + M.c2 * (rm - rp + r0));
}

// HERM off-diagonals a, b and u^2 = dt^2 (|a|^2 + |b|^2) / 4 at one point.
template <typename R>
__device__ __forceinline__ R herm_ab(const cx<R> &p, const cx<R> &z, const cx<R> &m, const Model<R> &M, cx<R> &a,
                                     cx<R> &b) {
    a = cfma(mk(M.c2, R(0)), conj(m) * z, mk(M.om_t, R(0)));
    b = cfma(mk(M.c2, R(0)), conj(z) * p, mk(M.om_t, R(0)));
    return R(0.25) * M.dt * M.dt * (abs2(a) + abs2(b));
}

// S = sinc(u) (sinhc in imaginary time) and C = cos(u) (cosh) from q = u^2:
// NT-term series, or (NT = 0) the 10-term series up to (pi/4)^2 and the
// library beyond.
template <typename R, int NT>
__device__ __forceinline__ void herm_sc(R q, int imag, R &S, R &C) {
    if (NT > 0) {
        S = imag ? series_q<R, false, 1, NT>(q) : series_q<R, true, 1, NT>(q);
        C = imag ? series_q<R, false, 0, NT>(q) : series_q<R, true, 0, NT>(q);
    } else if (q <= SeriesLimit<R>::q) {
        S = imag ? sinhc_q(q) : sinc_q(q);
        C = imag ? cosh_q(q) : cos_q(q);
    } else {
        const R u = sqrt_(q);
        if (imag) {
            S = sinh_(u) / u;
            C = cosh_(u);
        } else {
            R su, cu;
            sincos_(u, &su, &cu);
            S = su / u;
            C = cu;
        }
    }
}

template <typename R>
__device__ __forceinline__ void herm_apply(cx<R> &p, cx<R> &z, cx<R> &m, cx<R> a, cx<R> b, R S, R C,
                                           const Model<R> &M) {
    const cx<R> A0 = a * z, A1 = cfma(conj(a), p, b * m), A2 = conj(b) * z;
    const cx<R> B0 = a * A1, B1 = cfma(conj(a), A0, b * A2), B2 = conj(b) * A1;
    const R f = -M.dt * S * C;
    const R h = (M.imag ? R(0.5) : R(-0.5)) * M.dt * M.dt * S * S;
    if (M.imag) {
        p = p + f * A0 + h * B0;
        z = z + f * A1 + h * B1;
        m = m + f * A2 + h * B2;
    } else {
        p = p + f * mul_i(A0) + h * B0;
        z = z + f * mul_i(A1) + h * B1;
        m = m + f * mul_i(A2) + h * B2;
    }
}

// HERM with given off-diagonals a, b and q = u^2 = dt^2 (|a|^2 + |b|^2) / 4:
// the shortest series every lane of the wavefront allows.
template <typename R>
__device__ __forceinline__ void herm_with(cx<R> &p, cx<R> &z, cx<R> &m, cx<R> a, cx<R> b, R q, const Model<R> &M) {
    R S, C;
    if (__all(q <= R(SERIES_Q2))) herm_sc<R, 2>(q, M.imag, S, C);
    else if (__all(q <= R(SERIES_Q4))) herm_sc<R, 4>(q, M.imag, S, C);
    else herm_sc<R, 0>(q, M.imag, S, C);
    herm_apply(p, z, m, a, b, S, C, M);
}

template <typename R>
__device__ __forceinline__ void pointwise(cx<R> &p, cx<R> &z, cx<R> &m, R V, const Model<R> &M) {
    R th[3];
    calcnu_phases(p, z, m, V, M, th);
    if (M.imag) {
        p = exp_(-th[0]) * p;
        z = exp_(-th[1]) * z;
        m = exp_(-th[2]) * m;
    } else {
        R c, s;
        cos_sin(th[0], c, s);
        p = p * mk(c, -s);
        cos_sin(th[1], c, s);
        z = z * mk(c, -s);
        cos_sin(th[2], c, s);
        m = m * mk(c, -s);
    }
    cx<R> a, b;
    const R q = herm_ab(p, z, m, M, a, b);
    herm_with(p, z, m, a, b, q, M);
}

// Second-order pointwise stage over tau = M.dt (the opt-in Strang scheme,
// beyond the paper).  CALCNU and HERM take their coefficients frozen at
// their input, which is first order for c2 != 0; here the flow
// psi' = -k (Phi(psi) + A(psi)) psi is taken by the exponential midpoint
// rule: a predictor psi_m = HERM(tau/2) CALCNU(tau/2) psi (the sub-steps
// above over half the interval), Phi and A evaluated at psi_m, and
//   psi <- exp(-k tau/2 Phi_m) exp(-k tau A_m) exp(-k tau/2 Phi_m) psi
// (the two diagonal factors are the same numbers, computed once).
template <typename R>
__device__ __forceinline__ void pointwise2(cx<R> &p, cx<R> &z, cx<R> &m, R V, const Model<R> &M) {
    Model<R> Mh = M;
    Mh.dt = R(0.5) * M.dt;
    cx<R> mp = p, mz = z, mm = m;
    pointwise(mp, mz, mm, V, Mh);
    R th[3];
    calcnu_phases(mp, mz, mm, V, Mh, th);
    cx<R> a, b;
    const R q = herm_ab(mp, mz, mm, M, a, b);
    if (M.imag) {
        const R e0 = exp_(-th[0]), e1 = exp_(-th[1]), e2 = exp_(-th[2]);
        p = e0 * p;
        z = e1 * z;
        m = e2 * m;
        herm_with(p, z, m, a, b, q, M);
        p = e0 * p;
        z = e1 * z;
        m = e2 * m;
    } else {
        R c, s;
        cos_sin(th[0], c, s);
        const cx<R> e0 = mk(c, -s);
        cos_sin(th[1], c, s);
        const cx<R> e1 = mk(c, -s);
        cos_sin(th[2], c, s);
        const cx<R> e2 = mk(c, -s);
        p = p * e0;
        z = z * e1;
        m = m * e2;
        herm_with(p, z, m, a, b, q, M);
        p = p * e0;
        z = z * e1;
        m = m * e2;
    }
}

// -------------------------------------------------- chunked line solve ---
// Elimination coefficients of one line direction.  With o the
// off-diagonal of I + sT and m_i the Thomas pivots, c'_i = o / m_i and the
// forward sweep y_i = (r_i - o y_{i-1}) / m_i is y_i = c'_i (r_i/o - y_{i-1});
// the right-hand side is built already divided by o.  The pivots of a
// constant Toeplitz matrix converge: from index head on, c'_i is bitwise
// equal to cp_inf (the host finds head by running the recurrence in the
// table precision), so only the head is tabulated.
template <typename R> struct LineCoef {
    const cx<R> *cp;        // first head entries of c'_i
    const cx<R> *chunkA;    // per-chunk products of -c'_i
    const cx<R> *pw;        // 3 L products of -c'_i over a chunk (see ChunkCoef)
    cx<R> cp_inf;
    int head;               // >= 1
    int levels;             // scan levels: carries over more than 2^levels - 1
                            // chunks are below 2^-64 relative and dropped
};

// Coefficients of one chunk.  When the tabulated head is short (head <=
// min(L, CM), CM = 4 or 8: the pivots converge within a few points), c'_i is
// cp_inf for every entry except the first min(L, CM) entries of the chunk
// that starts the line: those few are selected per lane from wave-uniform
// table loads, and every other entry is the uniform stationary value, with no
// per-element select.  Otherwise (CM = 0) every lane reads its chunk's
// entries (clamped, unconditional loads) into registers.
//
// The carry fix-ups e_t = -c'_t e_{t-1} (forward) and e_t = -c'_t e_{t+1}
// (backward) of a chunk are products of the carry with partial products of
// -c'_i over the chunk.  For CM != 0 these are wave-uniform, so they are
// tabulated (pw, 3 L entries):
//   pw[t]       = prod_{s <= t} (-cp_inf)        forward, every chunk but the
//                                                first (whose carry is 0)
//   pw[L + t]   = prod_{s >= t} (-cp_inf)        backward, over L - t entries
//   pw[2 L + t] = prod_{s >= t} (-c'_s)          backward, the first chunk
// and every fix-up entry is one independent complex multiply-add.  A chunk
// shorter than L is the last of its line and receives a zero carry.
__host__ __device__ constexpr int coef_mode(int head, int L) {
    return L <= 2 ? 0 : head <= (L < 4 ? L : 4) ? 4 : head <= (L < 8 ? L : 8) ? 8 : 0;
}

template <typename R, int L, int CM> struct ChunkCoef {
    static constexpr int HM = L < CM ? L : CM;  // head <= HM
    const cx<R> *tab;
    const cx<R> *pw;
    cx<R> tail;
    int head;
    bool first;  // this lane's chunk starts at index 0
    __device__ __forceinline__ ChunkCoef(const LineCoef<R> &C, int start)
        : tab(C.cp), pw(C.pw), tail(C.cp_inf), head(C.head), first(start == 0) {}
    __device__ __forceinline__ cx<R> operator[](int t) const {
        if (t >= HM) return tail;  // t is a compile-time index: no select
        const cx<R> h = tab[t < head ? t : head - 1];  // uniform address
        return (first && t < head) ? h : tail;
    }
    __device__ __forceinline__ cx<R> fwd_pow(int t) const { return pw[t]; }
    __device__ __forceinline__ cx<R> bwd_pow(int t) const {
        if (t >= HM) return pw[L + t];
        return first ? pw[2 * L + t] : pw[L + t];
    }
};

template <typename R, int L> struct ChunkCoef<R, L, 0> {
    cx<R> v[L];
    __device__ __forceinline__ ChunkCoef(const LineCoef<R> &C, int start) {
#pragma unroll
        for (int t = 0; t < L; ++t) {
            const int i = start + t;
            const cx<R> x = C.cp[min(i, C.head - 1)];
            v[t] = i < C.head ? x : C.cp_inf;
        }
    }
    __device__ __forceinline__ cx<R> operator[](int t) const { return v[t]; }
};

// Forward sweep of one chunk with zero carry-in; r holds (I - sT)u / o on
// entry and the partial y on exit.  Returns the last y (0 if empty).
template <typename R, int L, typename CC>
__device__ __forceinline__ cx<R> fwd_local(cx<R> (&r)[L], int len, const CC &cpl) {
    cx<R> prev = czero<R>();
#pragma unroll
    for (int t = 0; t < L; ++t) {
        if (t < len) {
            prev = cpl[t] * (r[t] - prev);
            r[t] = prev;
        }
    }
    return prev;
}

// Adds the carried-in term: e_i = -c'_i e_{i-1}, e_{start-1} = carry.
template <typename R, int L, typename CC>
__device__ __forceinline__ void fwd_fix(cx<R> (&r)[L], int len, const CC &cpl, cx<R> carry) {
    cx<R> e = carry;
#pragma unroll
    for (int t = 0; t < L; ++t) {
        if (t < len) {
            e = czero<R>() - cpl[t] * e;
            r[t] = r[t] + e;
        }
    }
}
template <typename R, int L, int CM>
__device__ __forceinline__ void fwd_fix(cx<R> (&r)[L], int len, const ChunkCoef<R, L, CM> &cpl, cx<R> carry) {
    if constexpr (CM == 0) {
        fwd_fix<R, L, ChunkCoef<R, L, 0>>(r, len, cpl, carry);
    } else {
#pragma unroll
        for (int t = 0; t < L; ++t)
            if (t < len) r[t] = cfma(cpl.fwd_pow(t), carry, r[t]);
    }
}

// Back substitution x_i = y_i - c'_i x_{i+1} of one chunk with zero carry-in
// from the right.  Returns the first x (0 if empty).
template <typename R, int L, typename CC>
__device__ __forceinline__ cx<R> bwd_local(cx<R> (&r)[L], int len, const CC &cpl) {
#pragma unroll
    for (int t = L - 2; t >= 0; --t) {
        if (t + 1 < len) r[t] = r[t] - cpl[t] * r[t + 1];
    }
    return len > 0 ? r[0] : czero<R>();
}

template <typename R, int L, typename CC>
__device__ __forceinline__ void bwd_fix(cx<R> (&r)[L], int len, const CC &cpl, cx<R> carry) {
    cx<R> e = carry;
#pragma unroll
    for (int t = L - 1; t >= 0; --t) {
        if (t < len) {
            e = czero<R>() - cpl[t] * e;
            r[t] = r[t] + e;
        }
    }
}
template <typename R, int L, int CM>
__device__ __forceinline__ void bwd_fix(cx<R> (&r)[L], int len, const ChunkCoef<R, L, CM> &cpl, cx<R> carry) {
    if constexpr (CM == 0) {
        bwd_fix<R, L, ChunkCoef<R, L, 0>>(r, len, cpl, carry);
    } else {
#pragma unroll
        for (int t = 0; t < L; ++t)
            if (t < len) r[t] = cfma(cpl.bwd_pow(t), carry, r[t]);
    }
}

// The fix-ups of three lines with the same chunk coefficients, entry by
// entry (each tabulated product is loaded once for the three lines).
template <typename R, int L, int CM>
__device__ __forceinline__ void fwd_fix3(cx<R> (&r)[3][L], int len, const ChunkCoef<R, L, CM> &cpl,
                                         const cx<R> (&carry)[3]) {
    if constexpr (CM == 0) {
#pragma unroll
        for (int j = 0; j < 3; ++j) fwd_fix<R, L>(r[j], len, cpl, carry[j]);
    } else {
#pragma unroll
        for (int t = 0; t < L; ++t) {
            const cx<R> P = cpl.fwd_pow(t);
#pragma unroll
            for (int j = 0; j < 3; ++j)
                if (t < len) r[j][t] = cfma(P, carry[j], r[j][t]);
        }
    }
}
template <typename R, int L, int CM>
__device__ __forceinline__ void bwd_fix3(cx<R> (&r)[3][L], int len, const ChunkCoef<R, L, CM> &cpl,
                                         const cx<R> (&carry)[3]) {
    if constexpr (CM == 0) {
#pragma unroll
        for (int j = 0; j < 3; ++j) bwd_fix<R, L>(r[j], len, cpl, carry[j]);
    } else {
#pragma unroll
        for (int t = 0; t < L; ++t) {
            const cx<R> P = cpl.bwd_pow(t);
#pragma unroll
            for (int j = 0; j < 3; ++j)
                if (t < len) r[j][t] = cfma(P, carry[j], r[j][t]);
        }
    }
}

// Inclusive scan over the lanes lane, lane-STRIDE, lane-2*STRIDE, ... of the
// wavefront of the affine maps (A, B), over 2^levels - 1 predecessors:
// afterwards (A, B) maps the value before the window to the value after
// this lane's chunk (all earlier chunks contribute below rounding).
template <typename R, int STRIDE>
__device__ __forceinline__ void wave_scan_up(cx<R> &A, cx<R> &B, int levels) {
    const int lane = threadIdx.x & 63;
    int lv = 0;
#pragma unroll
    for (int d = STRIDE; d < 64; d <<= 1, ++lv) {
        if (lv >= levels) break;
        const cx<R> Ap = shfl_up(A, d), Bp = shfl_up(B, d);
        if (lane >= d) {
            B = cfma(A, Bp, B);
            A = A * Ap;
        }
    }
}

template <typename R, int STRIDE>
__device__ __forceinline__ void wave_scan_down(cx<R> &A, cx<R> &B, int levels) {
    const int lane = threadIdx.x & 63;
    int lv = 0;
#pragma unroll
    for (int d = STRIDE; d < 64; d <<= 1, ++lv) {
        if (lv >= levels) break;
        const cx<R> Ap = shfl_down(A, d), Bp = shfl_down(B, d);
        if (lane + d < 64) {
            B = cfma(A, Bp, B);
            A = A * Ap;
        }
    }
}

// The same with the lane's coefficients and chunk product already in registers.
template <typename R, int L>
__device__ __forceinline__ void solve_line_cached(cx<R> (&r)[L], int len, const ChunkCoef<R, L, 0> &cpl, cx<R> Ak,
                                                  int levels) {
    const int lane = threadIdx.x & 63;
    cx<R> A = Ak;
    cx<R> B = fwd_local<R, L>(r, len, cpl);
    wave_scan_up<R, 1>(A, B, levels);
    cx<R> carry = shfl_up(B, 1);
    if (lane == 0) carry = czero<R>();
    fwd_fix<R, L>(r, len, cpl, carry);
    A = Ak;
    B = bwd_local<R, L>(r, len, cpl);
    wave_scan_down<R, 1>(A, B, levels);
    carry = shfl_down(B, 1);
    if (lane == 63) carry = czero<R>();
    bwd_fix<R, L>(r, len, cpl, carry);
}

// Solves one line held by the 64 lanes of a wavefront (lane k owns
// [start, start+len)).
template <typename R, int L, int CM>
__device__ __forceinline__ void solve_line_wave(cx<R> (&r)[L], int start, int len, const LineCoef<R> &C) {
    const int lane = threadIdx.x & 63;
    const ChunkCoef<R, L, CM> cpl(C, start);
    const cx<R> Ak = C.chunkA[lane];
    cx<R> A = Ak;
    cx<R> B = fwd_local<R, L>(r, len, cpl);
    wave_scan_up<R, 1>(A, B, C.levels);
    cx<R> carry = shfl_up(B, 1);
    if (lane == 0) carry = czero<R>();
    fwd_fix<R, L>(r, len, cpl, carry);
    A = Ak;
    B = bwd_local<R, L>(r, len, cpl);
    wave_scan_down<R, 1>(A, B, C.levels);
    carry = shfl_down(B, 1);
    if (lane == 63) carry = czero<R>();
    bwd_fix<R, L>(r, len, cpl, carry);
}

// LDS index of point i with one padding slot after every chunk of L points,
// so that the 64 lanes reading "their" chunk hit distinct banks.
template <int L> __device__ __forceinline__ int sidx(int i) { return i + i / L; }
template <int L> __host__ __device__ constexpr int srow(int n) { return n + n / L + 1; }

// Right-hand side (I - sT) u of the x-line solve for component J over the
// lane's chunk, where u = psi + SO update:
//   u_J(i) = s_J(i) + ys_J(i) + sum_j' q[J][j'] (s_j'(i+1) - s_j'(i-1)),
// with s the staged row (zero outside [0, nx)) and ys optional precomputed
// y-derivative terms.  A sliding window reads every staged value once.
// (pat, qa, qb: the SO coefficient pattern of the x-derivative forms, as
// XArgs::sopat with 2 for the diagonal one; component J's terms j' = 0, 1, 2)
template <typename R, int L, int J>
__device__ __forceinline__ void build_rhs(const cx<R> *s, const cx<R> *ys, int ld, int nx, int start, int len,
                                          int pat, cx<R> qa, cx<R> qb, cx<R> rdiag,
                                          cx<R> (&r)[L]) {
    auto at = [&](int jp, int i) -> cx<R> {
        return (i >= 0 && i < nx) ? s[jp * ld + sidx<L>(i)] : czero<R>();
    };
    const bool use0 = (pat == 1 && J == 1) || (pat == 2 && J == 0), use1 = pat == 1 && J != 1,
               use2 = (pat == 1 && J == 1) || (pat == 2 && J == 2);
    const cx<R> q0 = J == 1 ? qb : qa, q1 = J == 0 ? qa : qb, q2 = J == 1 ? qa : qb;
    // window of the coupled components at i-1 and i+1, own component at i
    cx<R> m0{}, m1{}, m2{}, p0{}, p1{}, p2{}, c0{}, c1{}, c2{};
    auto load_win = [&](int i) {
        if (use0) { m0 = at(0, i - 1); c0 = at(0, i); p0 = at(0, i + 1); }
        if (use1) { m1 = at(1, i - 1); c1 = at(1, i); p1 = at(1, i + 1); }
        if (use2) { m2 = at(2, i - 1); c2 = at(2, i); p2 = at(2, i + 1); }
    };
    auto shift_win = [&](int i) {  // window moves from i-1 to i
        if (use0) { m0 = c0; c0 = p0; p0 = at(0, i + 1); }
        if (use1) { m1 = c1; c1 = p1; p1 = at(1, i + 1); }
        if (use2) { m2 = c2; c2 = p2; p2 = at(2, i + 1); }
    };
    auto u_at = [&](int i) -> cx<R> {
        if (i < 0 || i >= nx) return czero<R>();
        cx<R> v = at(J, i);
        if (ys) v = v + ys[J * ld + sidx<L>(i)];
        if (use0) v = cfma(q0, p0 - m0, v);
        if (use1) v = cfma(q1, p1 - m1, v);
        if (use2) v = cfma(q2, p2 - m2, v);
        return v;
    };
    if (len <= 0) {
#pragma unroll
        for (int t = 0; t < L; ++t) r[t] = czero<R>();
        return;
    }
    load_win(start - 1);
    cx<R> um = u_at(start - 1);
    shift_win(start);
    cx<R> uc = u_at(start);
#pragma unroll
    for (int t = 0; t < L; ++t) {
        if (t < len) {
            shift_win(start + t + 1);
            const cx<R> un = u_at(start + t + 1);
            r[t] = cn_rhs(rdiag, uc, um + un);
            um = uc;
            uc = un;
        } else {
            r[t] = czero<R>();
        }
    }
}

template <typename R, int L>
__device__ __forceinline__ void build_rhs_any(int J, const cx<R> *s, const cx<R> *ys, int ld, int nx, int start,
                                              int len, int pat, cx<R> qa, cx<R> qb, cx<R> rdiag,
                                              cx<R> (&r)[L]) {
    if (J == 0) build_rhs<R, L, 0>(s, ys, ld, nx, start, len, pat, qa, qb, rdiag, r);
    else if (J == 1) build_rhs<R, L, 1>(s, ys, ld, nx, start, len, pat, qa, qb, rdiag, r);
    else build_rhs<R, L, 2>(s, ys, ld, nx, start, len, pat, qa, qb, rdiag, r);
}

// ------------------------------------------------------------- x-pass ---
// ------------------------------------------------ RENORM on the device ---
// Rescaling factors of App. A: Eq. (DJ) keeps N = 1 and N_{+1} - N_{-1} = m,
// Eq. (DJ2) keeps N = 1 only.
struct RenormSpec {
    int fixed_m;   // 1: Eq. (DJ) (with the fall-backs), 0: Eq. (DJ2)
    double m;
    double dA;
};

__device__ __forceinline__ void renorm_factors(const RenormSpec &sp, const double N[3], double d[3],
                                               double *fallback) {
    const double Np = N[0], N0 = N[1], Nm = N[2];
    if (sp.fixed_m) {
        const double m = sp.m;
        if (fabs(m) < 1.0 && Np > 0.0 && Nm > 0.0) {
            const double d0 = sqrt(1.0 - m * m) / sqrt(N0 + sqrt(4.0 * (1.0 - m * m) * Np * Nm + m * m * N0 * N0));
            const double rp = 1.0 + m - d0 * d0 * N0, rm = 1.0 - m - d0 * d0 * N0;
            if (rp >= 0.0 && rm >= 0.0) {
                d[0] = sqrt(rp) / sqrt(2.0 * Np);
                d[1] = d0;
                d[2] = sqrt(rm) / sqrt(2.0 * Nm);
                *fallback = 0.0;
                return;
            }
        }
        *fallback = 1.0;
    }
    const double dd = 1.0 / sqrt(N0 + Np + Nm);
    d[0] = d[1] = d[2] = dd;
}

// Sums of per-tile |psi_j|^2 partials, stored [3][ntiles], by one whole
// wavefront in a fixed order: lane l adds tiles l, l + 64, l + 128, ... in
// turn, then the 64 lane sums are added pairwise (offsets 32, 16, ..., 1).
// Every caller (the finalize kernel, each x-pass workgroup) gets the same
// bits; the sums are in lane 0.
__device__ __forceinline__ void wave_tile_sums(const double *partials, int ntiles, double (&s)[3]) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        double t = 0.0;
        for (int q = lane; q < ntiles; q += 64) t += partials[(long long)j * ntiles + q];
        s[j] = t;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1)
#pragma unroll
        for (int j = 0; j < 3; ++j) s[j] += __shfl_down(s[j], d, 64);
}

// The three symmetrised lines of the unitary-SO scheme in device memory, for
// the x-pass variant whose scalar registers run short with them as kernel
// arguments (held for the whole pass, they spill).
template <typename R> struct UsoLines {
    LineCoef<R> cu[3];
    cx<R> rdiag_u[3];
};

template <typename R> struct XArgs {
    const cx<R> *src;          // state read (3 planes)
    cx<R> *dst;                // state written (may equal src)
    int nx, ny;
    long long plane;           // nx * ny
    R dx, dy, x0, y0;
    Model<R> m;
    const double *dscale;      // RENORM factors to apply first, or nullptr
    const double *rpart;       // or: the previous y-pass's tile partials [3][rntiles],
    int rntiles;               //     reduced here into the factors (rsp: the rule)
    RenormSpec rsp;
    int pointwise;             // 1: CALCNU + HERM in this pass (the second-order
                               //    kernels: the number of P2(dt/2) stages, 1 or 2)
    LineCoef<R> cx_;           // CN_x elimination coefficients (256 chunks of KM points)
    cx<R> rdiag;               // diagonal of (I - sT)/o (off-diagonal -1)
    cx<R> qx[9];               // SO: psi'_j += sum_j' qx[j][j'] (psi_j'(i+1) - psi_j'(i-1))
    unsigned qxmask;           // bit 3j+j' set where qx[j][j'] != 0
    // What the x-pass reads of qx (set by its launcher): the 2D grids' x
    // derivative SO terms (gamma p_x S_x, and the equal mixture's -gamma p_x
    // S_y) couple neighbouring components only, with qx[0][1] = qx[1][2] =: qa
    // and qx[1][0] = qx[2][1] =: qb (sopat 1); sopat 0: no SO terms.  Two
    // coefficients instead of nine keep the pass's scalar registers from
    // spilling.
    int sopat;
    cx<R> qa, qb;
    // Unitary-SO scheme (x-derivative SO forms; no qx terms then): the SO
    // term is solved together with CN_x.  In the eigenbasis of the SO spin
    // matrix component c is a tridiagonal Toeplitz system with off-diagonals
    // of equal modulus; the diagonal similarity by unit phases (the ramp of
    // line c) makes it symmetric, and it is solved like CN_x with the tables
    // cu[c] and rdiag_u[c].  Lines 0 and 2 (eigenvalues lambda and -lambda)
    // then have the same matrix: the kernels solve line 2 with line 0's
    // tables (cu[2] and rdiag_u[2] are left unread).  The basis change:
    // uso_in / uso_out.
    const cx<R> *ramp;         // [nx]: the ramp of line 0, or nullptr: the paper's scheme
    R rotr[9];                 // Wr (row j: component, column c: eigenvector)
    int rotp[3];               // the phase of row j: i^rotp[j]
    int rotphased;             // some rotp[j] != 0
    LineCoef<R> cu[3];
    cx<R> rdiag_u[3];
    const UsoLines<R> *ul;     // cu and rdiag_u again, in device memory (the Strang pass reads
                               // them there: its scalar registers run short)
    int uso_head;              // the longest of the three pivot heads (host: coefficient mode)
    int strang;                // 1: the second-order pointwise stages (with ramp)
    int rowgrp;                // > 0: workgroup b takes row (b / (8 g)) 8 g + (b mod 8) g + (b mod 8g) / 8
                               // (g = rowgrp): the 8 XCDs, which take workgroups round-robin, each
                               // get g adjacent rows of every block of 8 g; 0: row b
};

constexpr int XPASS_THREADS = 256;

// ------------------------------------------- unitary-SO basis change ---
// The eigenvector matrix of the SO spin matrix (row j: component, column c:
// eigenvector) is W = diag(i^p_j) Wr with Wr real, and the eigenvalues are
// (lambda, 0, -lambda), so the phase ramps of lines 1 and 2 are 1 and the
// conjugate of line 0's (the host builds them so).  Into the symmetrised
// basis: w_c = conj(ramp_c) sum_j Wr[j][c] i^-p_j v_j; back:
// v_j = i^p_j sum_c Wr[j][c] ramp_c w_c.  Wr holds real numbers, so each
// term is two multiply-adds.
template <typename R> __device__ __forceinline__ cx<R> mul_ipow(cx<R> v, int k) {  // v i^k
    switch (k & 3) {
    case 1: return mk(-v.y, v.x);
    case 2: return mk(-v.x, -v.y);
    case 3: return mk(v.y, -v.x);
    default: return v;
    }
}
template <typename R> __device__ __forceinline__ cx<R> uso_ramp_line(int c, cx<R> ramp0) {
    return c == 0 ? ramp0 : c == 1 ? mk(R(1), R(0)) : conj(ramp0);
}
template <typename R, typename A> __device__ __forceinline__ void uso_in(const A &a, cx<R> (&v)[3], cx<R> ramp0) {
    if (a.rotphased)
#pragma unroll
        for (int j = 0; j < 3; ++j) v[j] = mul_ipow(v[j], 4 - a.rotp[j]);
    cx<R> w[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) w[c] = a.rotr[c] * v[0] + a.rotr[3 + c] * v[1] + a.rotr[6 + c] * v[2];
    v[0] = conj(ramp0) * w[0];
    v[1] = w[1];
    v[2] = ramp0 * w[2];
}
template <typename R, typename A> __device__ __forceinline__ void uso_rotate_out(const A &a, cx<R> (&w)[3]) {
    cx<R> v[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) v[j] = a.rotr[3 * j] * w[0] + a.rotr[3 * j + 1] * w[1] + a.rotr[3 * j + 2] * w[2];
    if (a.rotphased)
#pragma unroll
        for (int j = 0; j < 3; ++j) v[j] = mul_ipow(v[j], a.rotp[j]);
#pragma unroll
    for (int j = 0; j < 3; ++j) w[j] = v[j];
}
template <typename R, typename A> __device__ __forceinline__ void uso_out(const A &a, cx<R> (&w)[3], cx<R> ramp0) {
    w[0] = ramp0 * w[0];
    w[2] = conj(ramp0) * w[2];
    uso_rotate_out(a, w);
}
// 1D kernel: wavefronts 0-2 solve the three component lines; all of them
// share the pointwise work (more wavefronts where the chunk registers allow)
__host__ __device__ constexpr int step1d_threads(int L) { return L >= 16 ? 256 : 512; }

// Whole-wavefront rotations by one lane (DPP wave_ror:1 / wave_rol:1):
// ror1 gives lane l the value of lane l-1 (lane 0 gets lane 63), rol1 the
// value of lane l+1 (lane 63 gets lane 0).  Every lane must execute them.
__device__ __forceinline__ unsigned dpp_ror1(unsigned v) { return __builtin_amdgcn_update_dpp(0u, v, 0x13C, 0xF, 0xF, false); }
__device__ __forceinline__ unsigned dpp_rol1(unsigned v) { return __builtin_amdgcn_update_dpp(0u, v, 0x134, 0xF, 0xF, false); }
__device__ __forceinline__ double ror1(double x) {
    const unsigned long long u = __double_as_longlong(x);
    const unsigned lo = dpp_ror1((unsigned)u), hi = dpp_ror1((unsigned)(u >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ double rol1(double x) {
    const unsigned long long u = __double_as_longlong(x);
    const unsigned lo = dpp_rol1((unsigned)u), hi = dpp_rol1((unsigned)(u >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ float ror1(float x) { return __uint_as_float(dpp_ror1(__float_as_uint(x))); }
__device__ __forceinline__ float rol1(float x) { return __uint_as_float(dpp_rol1(__float_as_uint(x))); }
template <typename R> __device__ __forceinline__ cx<R> ror1(cx<R> v) { return {ror1(v.x), ror1(v.y)}; }
template <typename R> __device__ __forceinline__ cx<R> rol1(cx<R> v) { return {rol1(v.x), rol1(v.y)}; }

// Three affine-map scans (one per component) over the lanes of a wavefront,
// interleaved level by level; see wave_scan_up / wave_scan_down.
template <typename R>
__device__ __forceinline__ void wave_scan_up3(cx<R> (&A)[3], cx<R> (&B)[3], int levels) {
    const int lane = threadIdx.x & 63;
    int lv = 0;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1, ++lv) {
        if (lv >= levels) break;
        cx<R> Ap[3], Bp[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            Ap[j] = shfl_up(A[j], d);
            Bp[j] = shfl_up(B[j], d);
        }
        if (lane >= d) {
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                B[j] = cfma(A[j], Bp[j], B[j]);
                A[j] = A[j] * Ap[j];
            }
        }
    }
}

template <typename R>
__device__ __forceinline__ void wave_scan_down3(cx<R> (&A)[3], cx<R> (&B)[3], int levels) {
    const int lane = threadIdx.x & 63;
    int lv = 0;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1, ++lv) {
        if (lv >= levels) break;
        cx<R> Ap[3], Bp[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            Ap[j] = shfl_down(A[j], d);
            Bp[j] = shfl_down(B[j], d);
        }
        if (lane + d < 64) {
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                B[j] = cfma(A[j], Bp[j], B[j]);
                A[j] = A[j] * Ap[j];
            }
        }
    }
}

// x-pass: one workgroup of 4 wavefronts per row.  Thread t owns the KM
// consecutive points t*KM .. t*KM + KM - 1 of all three components from the
// loads to the stores, so the stencil neighbours are in its own registers
// except at its two ends: the previous thread's last and the next thread's
// first value come by DPP whole-wave rotations, and across wavefronts
// through a two-value LDS exchange.  In this layout the pass applies the
// previous RENORM, CALCNU and HERM, the SO update and the Crank-Nicolson
// right-hand side, and solves the three lines: the row is 256 chunks of KM
// points, one per thread; each thread eliminates its chunk for the three
// components (three independent recurrences), the chunk maps are scanned
// within each wavefront and carried across the 4 wavefronts through LDS, and
// each thread applies its carry fix-ups and stores its points.  FULL: the
// row has exactly 256 KM points, so no point needs a range check.  (The SO
// forms with y derivatives come here with their SO update already applied,
// from pso_kernel, and no SO terms.)
template <typename R, int KM> struct XShared {
    double d[3];                       // RENORM factors
    cx<R> E[2 * 24];                   // edges: [round][4 waves][2 ends][3 comps]
    cx<R> scA[2][4][3], scB[2][4][3];  // wavefront maps: [sweep][wave][comp]
    cx<R> xch[4][KM > 1 ? 64 * KM + 64 : 1];  // per-wavefront store line (see store_row)
};

// Stores of one row.  Wavefront w holds the 64 KM consecutive points
// 64 KM w + p, p < 64 KM, of the row in the blocked order (lane l: points
// p = KM l + m).  The stores are coalesced (store k of lane l: point
// p = 64 k + l): the blocked values pass through the wavefront's own LDS
// line, one padding slot after every KM points so that the blocked accesses
// (stride KM + 1 slots) spread over the banks.  A wavefront's LDS operations
// complete in issue order, so a wavefront-level compiler barrier orders
// them.  All three components are read back before the first store is
// issued (a store's data registers must not be reused while it is in
// flight).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Complex values moved as two-element vectors (first-class values, so that
// the copies stay in registers).
template <typename R> using vec2 = R __attribute__((ext_vector_type(2)));
template <typename R> __device__ __forceinline__ void put2(cx<R> *p, cx<R> v) {
    *reinterpret_cast<vec2<R> *>(p) = vec2<R>{v.x, v.y};
}
template <typename R> __device__ __forceinline__ cx<R> get2(const cx<R> *p) {
    const vec2<R> t = *reinterpret_cast<const vec2<R> *>(p);
    return cx<R>{t.x, t.y};
}

// blocked b[m] (point KM lane + m) -> coalesced c[k] (point 64 k + lane)
template <typename R, int KM>
__device__ __forceinline__ void wave_exchange(cx<R> *line, int lane, const cx<R> (&b)[KM], cx<R> (&c)[KM]) {
#pragma unroll
    for (int m = 0; m < KM; ++m) {
        const int p = KM * lane + m;
        put2(line + p + p / KM, b[m]);
    }
    wave_lds_sync();
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        const int p = 64 * k + lane;
        c[k] = get2(line + p + p / KM);
    }
    wave_lds_sync();
}

template <typename R, int KM, bool FULL>
__device__ __forceinline__ void store_row(cx<R> *dst, long long plane, int nx, const cx<R> (&r)[3][KM],
                                          cx<R> *line, int w) {
    const int lane = (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
    const int wbase = 64 * KM * w;
    if constexpr (KM == 1) {
#pragma unroll
        for (int j = 0; j < 3; ++j)
            if (FULL || wbase + lane < nx) dst[j * plane + wbase + lane] = r[j][0];
    } else {
        cx<R> c0[KM], c1[KM], c2[KM];
        wave_exchange<R, KM>(line, lane, r[0], c0);
        wave_exchange<R, KM>(line, lane, r[1], c1);
        wave_exchange<R, KM>(line, lane, r[2], c2);
#pragma unroll
        for (int k = 0; k < KM; ++k) {
            const int i = wbase + 64 * k + lane;
            if (FULL || i < nx) {
                put2(dst + i, c0[k]);
                put2(dst + plane + i, c1[k]);
                put2(dst + 2 * plane + i, c2[k]);
            }
        }
    }
}

// Everything after the loads, for one row whose KM points per thread are in
// v (zero beyond nx).
template <typename R, int KM, int CM, bool FULL, bool USO, bool P2>
__device__ __forceinline__ void xpass_row(const XArgs<R> &a, int row, cx<R> (&v)[3][KM], XShared<R, KM> &sh) {
    cx<R> *E = sh.E;
    auto &scA = sh.scA;
    auto &scB = sh.scB;
    const int nx = FULL ? XPASS_THREADS * KM : a.nx;
    const int tid = threadIdx.x, w = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const int i0 = tid * KM;  // this thread's points: i0 .. i0 + KM - 1
    const long long roff = (long long)row * nx;

    // ---- RENORM scale, CALCNU + HERM
    if (__builtin_expect(a.rpart != nullptr, 0)) {  // (measured: the layout keeps the real-time pass as fast)
        // the factors from the previous step's tile partials: the same
        // fixed-order sums as renorm_finalize_kernel, in every workgroup
        // (wavefront 0; the others' loads are in flight meanwhile)
        if (w == 0) {
            double sum[3];
            wave_tile_sums(a.rpart, a.rntiles, sum);
            if (lane == 0) {
                const double N[3] = {sum[0] * a.rsp.dA, sum[1] * a.rsp.dA, sum[2] * a.rsp.dA};
                double fb = 0.0;
                renorm_factors(a.rsp, N, sh.d, &fb);
            }
        }
        __syncthreads();
    }
    {
        const bool scale = a.dscale || a.rpart;
        const double *ds = a.rpart ? sh.d : a.dscale;
        R d0 = R(1), d1 = R(1), d2 = R(1);
        if (scale) {
            d0 = R(ds[0]);
            d1 = R(ds[1]);
            d2 = R(ds[2]);
        }
        const R yv = a.y0 + R(row) * a.dy;
        const R vy = R(0.5) * a.m.kappa2 * yv * yv;
#pragma unroll
        for (int k = 0; k < KM; ++k) {
            const int i = i0 + k;
            if (FULL || i < nx) {
                if (scale) {
                    v[0][k] = d0 * v[0][k];
                    v[1][k] = d1 * v[1][k];
                    v[2][k] = d2 * v[2][k];
                }
                if constexpr (P2) {
                    // a.pointwise stages P2(dt/2): the previous step's last
                    // and this step's first, or this step's first only
                    const R xv = a.x0 + R(i) * a.dx;
                    Model<R> Mt = a.m;
                    Mt.dt = R(0.5) * a.m.dt;
                    for (int rep = 0; rep < a.pointwise; ++rep)
                        pointwise2(v[0][k], v[1][k], v[2][k], R(0.5) * xv * xv + vy, Mt);
                } else if (a.pointwise) {
                    const R xv = a.x0 + R(i) * a.dx;
                    pointwise(v[0][k], v[1][k], v[2][k], R(0.5) * xv * xv + vy, a.m);
                }
            }
        }
    }
    if constexpr (USO) {
        // into the symmetrised eigenbasis
#pragma unroll
        for (int k = 0; k < KM; ++k) {
            const int i = i0 + k;
            if (FULL || i < nx) {
                cx<R> w[3] = {v[0][k], v[1][k], v[2][k]};
                uso_in(a, w, a.ramp[i]);
#pragma unroll
                for (int c = 0; c < 3; ++c) v[c][k] = w[c];
            }
        }
    }

    // values just outside this thread's points: the previous thread's last
    // and the next thread's first (DPP within the wavefront, LDS between)
    auto exchange_edges = [&](cx<R> (&x)[3][KM], int round) {
        cx<R> *Er = E + round * 24;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            if (lane == 0) Er[(w * 2 + 0) * 3 + j] = x[j][0];
            if (lane == 63) Er[(w * 2 + 1) * 3 + j] = x[j][KM - 1];
        }
    };
    auto outer = [&](cx<R> (&x)[3][KM], int round, int j, cx<R> &before, cx<R> &after) {
        const cx<R> *Er = E + round * 24;
        before = ror1(x[j][KM - 1]);
        after = rol1(x[j][0]);
        if (lane == 0) before = w > 0 ? Er[((w - 1) * 2 + 1) * 3 + j] : czero<R>();
        if (lane == 63) after = w < 3 ? Er[((w + 1) * 2 + 0) * 3 + j] : czero<R>();
    };

    // ---- SO update u = v + q (v(i+1) - v(i-1))
    exchange_edges(v, 0);
    __syncthreads();
    cx<R> u[3][KM];
    cx<R> vb[3], va[3];
#pragma unroll
    for (int jp = 0; jp < 3; ++jp) outer(v, 0, jp, vb[jp], va[jp]);
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int k = 0; k < KM; ++k) u[j][k] = v[j][k];
    // the terms of each point in the order j' = 0, 1, 2 of the sum over j'
    if (a.sopat != 0) {
#pragma unroll
        for (int k = 0; k < KM; ++k) {
            cx<R> d[3];  // psi_j'(i+1) - psi_j'(i-1)
#pragma unroll
            for (int jp = 0; jp < 3; ++jp) {
                const cx<R> pv = k > 0 ? v[jp][k > 0 ? k - 1 : 0] : vb[jp];
                const cx<R> nv = k + 1 < KM ? v[jp][k + 1 < KM ? k + 1 : 0] : va[jp];
                d[jp] = nv - pv;
            }
            u[0][k] = cfma(a.qa, d[1], u[0][k]);
            u[1][k] = cfma(a.qa, d[2], cfma(a.qb, d[0], u[1][k]));
            u[2][k] = cfma(a.qb, d[1], u[2][k]);
        }
    }
#pragma unroll
    for (int k = 0; k < KM; ++k)
        if (!FULL && i0 + k >= nx)
#pragma unroll
            for (int j = 0; j < 3; ++j) u[j][k] = czero<R>();

    // ---- right-hand side (I - sT) u / o; without SO terms (the y-derivative
    // forms after their pointwise + SO pass, no coupling) u is v, whose outer
    // values are at hand: no second exchange
    cx<R> ub[3], ua[3];  // u just before and just after this thread's points
    if (!USO && a.sopat == 0) {  // (the unitary-SO pass keeps the exchange: it measured faster so)
#pragma unroll
        for (int jj = 0; jj < 3; ++jj) {
            ub[jj] = vb[jj];
            ua[jj] = va[jj];
        }
    } else {
        exchange_edges(u, 1);
        __syncthreads();
#pragma unroll
        for (int jj = 0; jj < 3; ++jj) outer(u, 1, jj, ub[jj], ua[jj]);
    }
    cx<R> r[3][KM];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
#pragma unroll
        for (int k = 0; k < KM; ++k) {
            const cx<R> pu = k > 0 ? u[j][k > 0 ? k - 1 : 0] : ub[j];
            const cx<R> nu = k + 1 < KM ? u[j][k + 1 < KM ? k + 1 : 0] : ua[j];
            r[j][k] = (FULL || i0 + k < nx) ? cn_rhs(USO ? (P2 ? a.ul->rdiag_u[j & 1] : a.rdiag_u[j & 1]) : a.rdiag, u[j][k], pu + nu)
                                            : czero<R>();
        }
    }

    // ---- Crank-Nicolson solve of the three lines, chunk = this thread's points
    const int len = FULL ? KM : max(0, min(KM, nx - i0));
    // one coefficient set for the three lines, or (USO) one per line
    // the unitary-SO lines' coefficients (the Strang pass reads them from memory)
    const LineCoef<R> *ucf = P2 ? a.ul->cu : a.cu;
    const ChunkCoef<R, KM, CM> cpl(USO ? ucf[0] : a.cx_, i0);
    const ChunkCoef<R, KM, CM> cpl1(USO ? ucf[1] : a.cx_, i0);
    const ChunkCoef<R, KM, CM> cpl2(USO ? ucf[0] : a.cx_, i0);  // (USO: line 2 has line 0's matrix)
    auto coef = [&](int j) -> const ChunkCoef<R, KM, CM> & { return j == 0 ? cpl : j == 1 ? cpl1 : cpl2; };
    const cx<R> Ak = a.cx_.chunkA[tid];
    const int levels = USO ? ucf[0].levels : a.cx_.levels;  // (USO: the host gives the three the same)
    cx<R> A[3], B[3];
    // forward sweep: chunk eliminations, scan, carries across wavefronts
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        A[j] = USO ? ucf[j & 1].chunkA[tid] : Ak;
        B[j] = fwd_local<R, KM>(r[j], len, USO ? coef(j) : cpl);
    }
    wave_scan_up3<R>(A, B, levels);
    if (lane == 63) {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            scA[0][w][j] = A[j];
            scB[0][w][j] = B[j];
        }
    }
    __syncthreads();
    // carry into this wavefront: the maps of the wavefronts before it, in
    // order, the three components' entries of one wavefront read together
    cx<R> carry[3] = {czero<R>(), czero<R>(), czero<R>()};
    for (int q = 0; q < w; ++q) {
        cx<R> mA[3], mB[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            mA[j] = scA[0][q][j];
            mB[j] = scB[0][q][j];
        }
#pragma unroll
        for (int j = 0; j < 3; ++j) carry[j] = cfma(mA[j], carry[j], mB[j]);
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const cx<R> prev = shfl_up(cfma(A[j], carry[j], B[j]), 1);
        if (lane >= 1) carry[j] = prev;
    }
    if constexpr (USO) {
#pragma unroll
        for (int j = 0; j < 3; ++j) fwd_fix<R, KM>(r[j], len, coef(j), carry[j]);
    } else {
        fwd_fix3<R, KM>(r, len, cpl, carry);
    }
    // back substitution: chunk sweeps, reverse scan, carries
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        A[j] = USO ? ucf[j & 1].chunkA[tid] : Ak;
        B[j] = bwd_local<R, KM>(r[j], len, USO ? coef(j) : cpl);
    }
    wave_scan_down3<R>(A, B, levels);
    if (lane == 0) {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            scA[1][w][j] = A[j];
            scB[1][w][j] = B[j];
        }
    }
    __syncthreads();
    cx<R> *dst = a.dst + roff;
#pragma unroll
    for (int j = 0; j < 3; ++j) carry[j] = czero<R>();
    for (int q = 3; q > w; --q) {
        cx<R> mA[3], mB[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            mA[j] = scA[1][q][j];
            mB[j] = scB[1][q][j];
        }
#pragma unroll
        for (int j = 0; j < 3; ++j) carry[j] = cfma(mA[j], carry[j], mB[j]);
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const cx<R> next = shfl_down(cfma(A[j], carry[j], B[j]), 1);
        if (lane < 63) carry[j] = next;
    }
    if constexpr (USO) {
#pragma unroll
        for (int j = 0; j < 3; ++j) bwd_fix<R, KM>(r[j], len, coef(j), carry[j]);
        // back from the symmetrised eigenbasis
#pragma unroll
        for (int k = 0; k < KM; ++k) {
            const int i = i0 + k;
            if (FULL || i < nx) {
                cx<R> w[3] = {r[0][k], r[1][k], r[2][k]};
                uso_out(a, w, a.ramp[i]);
#pragma unroll
                for (int j = 0; j < 3; ++j) r[j][k] = w[j];
            }
        }
    } else {
        bwd_fix3<R, KM>(r, len, cpl, carry);
    }
    store_row<R, KM, FULL>(dst, a.plane, nx, r, sh.xch[w], w);
}

// (The unitary-SO form holds three coefficient sets per thread: with
// per-lane tables (CM = 0), or from 8 points per thread on, it takes the
// registers of 2 wavefronts per SIMD; with 4 points and tabulated fix-ups it
// keeps 4, which measured faster at 1024^2 than 2 without register spills:
// 36.6 against 39.4 us.)
template <typename R, int KM, int CM, bool FULL, bool USO = false, bool P2 = false>
__global__ void __launch_bounds__(XPASS_THREADS)
__attribute__((amdgpu_waves_per_eu(P2 ? (KM <= 4 ? 2 : 1)
                                   : USO ? (KM <= 1 || (KM <= 4 && CM != 0) ? 4 : 2)
                                         : (KM <= 4 ? 4 : 1))))
xpass_kernel(XArgs<R> a) {
    __shared__ XShared<R, KM> sh;
    const int nx = FULL ? XPASS_THREADS * KM : a.nx;
    int row = blockIdx.x;
    if (a.rowgrp > 0) {
        const int g = a.rowgrp, blk = 8 * g;
        if (row < (int)gridDim.x / blk * blk) row = row / blk * blk + (row % blk % 8) * g + row % blk / 8;
    }
    const int i0 = threadIdx.x * KM;
    const cx<R> *src = a.src + (long long)row * nx;
    cx<R> v[3][KM];
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        const int i = i0 + k;
#pragma unroll
        for (int j = 0; j < 3; ++j) v[j][k] = (FULL || i < nx) ? src[j * a.plane + i] : czero<R>();
    }
    xpass_row<R, KM, CM, FULL, USO, P2>(a, row, v, sh);
}

// ------------------------------------------------------------- y-pass ---
template <typename R> struct YArgs {
    cx<R> *psi;                // state, updated in place
    int nx, ny;
    long long plane;
    LineCoef<R> cy;            // CN_y elimination coefficients (blockDim/TX chunks)
    cx<R> rdiag;
    double *norm_partials;     // [3][gridDim.x] sums of |psi|^2, or nullptr
};

constexpr int YPASS_MAX_THREADS = 512;
constexpr int YPASS_MAX_WAVES = YPASS_MAX_THREADS / 64;

// Loads, right-hand side, elimination and chunk scans of one y-pass lane
// (FULL: the lane holds L rows and its column is valid).
template <typename R, int L, int TX, int CM, bool FULL>
__device__ __forceinline__ void ypass_solve(const YArgs<R> &a, const cx<R> *col, int start, int len, int k, int c,
                                            int lane, int wave, int nw, cx<R> (&r)[L],
                                            cx<R> (&scA)[2][YPASS_MAX_WAVES][TX],
                                            cx<R> (&scB)[2][YPASS_MAX_WAVES][TX]) {
    const int nx = a.nx, ny = a.ny;
    if (FULL) len = L;
    cx<R> f[L];
#pragma unroll
    for (int t = 0; t < L; ++t) f[t] = (FULL || t < len) ? col[(long long)(start + t) * nx] : czero<R>();
    // The rows just outside the chunk are the last row of chunk k - 1 and the
    // first row of chunk k + 1, held by lanes tid - TX and tid + TX (whenever
    // they are needed, those chunks are full and their lanes launched: the
    // workgroup is whole wavefronts of chunks covering ny).  Only the lanes at
    // the ends of a wavefront load them, issued with the chunk's own loads.
    const bool hl = len > 0 && start >= 1, hr = len > 0 && start + len < ny;
    const cx<R> el = (hl && lane < TX) ? col[(long long)(start - 1) * nx] : czero<R>();
    const cx<R> er = (hr && lane >= 64 - TX) ? col[(long long)(start + len) * nx] : czero<R>();
    const cx<R> up = shfl_up(f[L - 1], TX), dn = shfl_down(f[0], TX);
    const cx<R> fl = hl ? (lane >= TX ? up : el) : czero<R>();
    const cx<R> fr = hr ? (lane < 64 - TX ? dn : er) : czero<R>();
#pragma unroll
    for (int t = 0; t < L; ++t) {
        if (FULL || t < len) {
            const cx<R> left = t == 0 ? fl : f[t > 0 ? t - 1 : 0];
            const cx<R> right = FULL ? (t + 1 < L ? f[t + 1 < L ? t + 1 : 0] : fr)
                                     : ((t + 1 < L && t + 1 < len) ? f[t + 1 < L ? t + 1 : 0] : fr);
            r[t] = cn_rhs(a.rdiag, f[t], left + right);
        } else {
            r[t] = czero<R>();
        }
    }

    const ChunkCoef<R, L, CM> cpl(a.cy, start);
    const cx<R> Ak = a.cy.chunkA[k];
    // forward sweep and its scan over the chunks of each column
    cx<R> A = Ak;
    cx<R> B = fwd_local<R, L>(r, len, cpl);
    wave_scan_up<R, TX>(A, B, a.cy.levels);
    if (lane >= 64 - TX) {
        scA[0][wave][c] = A;
        scB[0][wave][c] = B;
    }
    __syncthreads();
    cx<R> carry = czero<R>();
    for (int w = 0; w < wave; ++w) carry = cfma(scA[0][w][c], carry, scB[0][w][c]);
    {
        const cx<R> incl = cfma(A, carry, B);
        const cx<R> prev = shfl_up(incl, TX);
        if (lane >= TX) carry = prev;
    }
    fwd_fix<R, L>(r, len, cpl, carry);

    // back substitution and its reverse scan
    A = Ak;
    B = bwd_local<R, L>(r, len, cpl);
    wave_scan_down<R, TX>(A, B, a.cy.levels);
    if (lane < TX) {
        scA[1][wave][c] = A;
        scB[1][wave][c] = B;
    }
    __syncthreads();
    carry = czero<R>();
    for (int w = nw - 1; w > wave; --w) carry = cfma(scA[1][w][c], carry, scB[1][w][c]);
    {
        const cx<R> incl = cfma(A, carry, B);
        const cx<R> next = shfl_down(incl, TX);
        if (lane < 64 - TX) carry = next;
    }
    bwd_fix<R, L>(r, len, cpl, carry);
}

// Workgroup: TX adjacent columns x P chunks of L rows (blockDim = TX * P);
// lane tid holds column tid % TX, chunk tid / TX.  grid = (ceil(nx/TX), 3):
// one workgroup per (tile, component).
template <typename R, int L, int TX, int CM>
__global__ void __launch_bounds__(YPASS_MAX_THREADS) ypass_kernel(YArgs<R> a) {
    __shared__ cx<R> scA[2][YPASS_MAX_WAVES][TX], scB[2][YPASS_MAX_WAVES][TX];
    __shared__ double red[YPASS_MAX_WAVES];
    const int nx = a.nx, ny = a.ny;
    // Workgroups are dispatched round-robin over the 8 XCDs; map them so that
    // each XCD takes a contiguous range of tiles, keeping the two tiles that
    // share a 128-byte line in one L2.
    const int ntx = gridDim.x;
    const int nb = ntx * gridDim.y;
    const int b = blockIdx.x + ntx * blockIdx.y;
    const int tile = (nb % 8 == 0) ? (b % 8) * (nb / 8) + b / 8 : b;
    const int j = tile / ntx, tx = tile % ntx;
    const int tid = threadIdx.x, c = tid % TX, k = tid / TX;
    const int lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
    const int x = tx * TX + c;
    const bool valid = x < nx;
    const int start = k * L;
    const int len = valid ? max(0, min(L, ny - start)) : 0;
    cx<R> *col = a.psi + j * a.plane + (valid ? x : 0);

    // every chunk full and every column valid: loads, right-hand side and
    // sweeps without per-element predication (uniform branch)
    const bool full = (ny == (int)(blockDim.x / TX) * L) && (nx % TX == 0);
    cx<R> r[L];
    if (full) ypass_solve<R, L, TX, CM, true>(a, col, start, L, k, c, lane, wave, nw, r, scA, scB);
    else ypass_solve<R, L, TX, CM, false>(a, col, start, len, k, c, lane, wave, nw, r, scA, scB);

    double nrm = 0.0;
#pragma unroll
    for (int t = 0; t < L; ++t) {
        if (t < len) {
            col[(long long)(start + t) * nx] = r[t];
            nrm += (double)abs2(r[t]);
        }
    }
    if (a.norm_partials) {
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) nrm += __shfl_down(nrm, d, 64);
        if (lane == 0) red[wave] = nrm;
        __syncthreads();
        if (tid == 0) {
            double t = 0.0;
            for (int w = 0; w < nw; ++w) t += red[w];
            a.norm_partials[(long long)j * ntx + tx] = t;
        }
    }
}

// -------------------------------------- second-order pointwise pass ---
// The closing stage P2 over m.dt of a step of the opt-in Strang scheme
// (after its y-pass), in place, from psi (RENORM factors dscale applied
// first when given); with norm_partials, each workgroup's sums of |psi_j|^2
// of the result in norm_partials[j * gridDim.x + block] (for the RENORM that
// follows).
template <typename R> struct PArgs {
    cx<R> *psi;
    int nx, ny;
    long long plane;
    R dx, dy, x0, y0;
    Model<R> m;
    const double *dscale;
    double *norm_partials;
};

template <typename R>
__global__ void __launch_bounds__(256) pointwise_kernel(PArgs<R> a) {
    const long long n = a.plane;
    double nrm[3] = {0.0, 0.0, 0.0};
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (long long)gridDim.x * blockDim.x) {
        const int ix = (int)(q % a.nx), iy = (int)(q / a.nx);
        cx<R> p = a.psi[q], z = a.psi[n + q], m = a.psi[2 * n + q];
        if (a.dscale) {
            p = R(a.dscale[0]) * p;
            z = R(a.dscale[1]) * z;
            m = R(a.dscale[2]) * m;
        }
        const R xv = a.x0 + R(ix) * a.dx, yv = a.y0 + R(iy) * a.dy;
        pointwise2(p, z, m, R(0.5) * (xv * xv + a.m.kappa2 * yv * yv), a.m);
        a.psi[q] = p;
        a.psi[n + q] = z;
        a.psi[2 * n + q] = m;
        nrm[0] += (double)abs2(p);
        nrm[1] += (double)abs2(z);
        nrm[2] += (double)abs2(m);
    }
    if (a.norm_partials) {
        __shared__ double red[3][4];
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            double t = nrm[j];
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) t += __shfl_down(t, d, 64);
            if (lane == 0) red[j][wave] = t;
        }
        __syncthreads();
        if (threadIdx.x < 3) {
            const int j = threadIdx.x;
            a.norm_partials[(long long)j * gridDim.x + blockIdx.x] = red[j][0] + red[j][1] + red[j][2] + red[j][3];
        }
    }
}

// ------------------------------- pointwise + SO pass (y-derivative SO) ---
// The SO update of the couplings with y derivatives (Rashba, Dresselhaus)
// takes the neighbours of a point in y after their CALCNU and HERM, which a
// row-per-workgroup x-pass does not hold.  This pass takes the state through
// RENORM scale, CALCNU, HERM and the whole SO update psi - k dt H_SO psi
// (central differences, zero ghosts beyond the grid; per point the x terms,
// then the y terms, in the order of the x-pass) into a second buffer, and
// the x-pass then runs CN_x on that buffer with neither.
//
// One workgroup per tile of 64 columns and PSO_TY = PSO_WAVES * PSO_RPW
// rows: wavefront w owns PSO_RPW consecutive rows of the tile and lane l
// column l.  x neighbours come from the adjacent lanes (DPP), y neighbours
// from the wavefront's own registers or, for its first and last row, from
// the adjacent wavefronts through LDS.  The pointwise values just outside
// the tile are recomputed (halo): the row above by wavefront 0, the row
// below by the last wavefront, the columns left and right by wavefront 1.
template <typename R> struct SOArgs {
    const cx<R> *src;          // state (read only)
    cx<R> *dst;                // the state after SO (another buffer)
    int nx, ny;
    long long plane;
    R dx, dy, x0, y0;
    Model<R> m;
    const double *dscale;      // RENORM factors to apply first, or nullptr
    cx<R> qx[9], qy[9];        // as in XArgs
    unsigned qxmask, qymask;
    // what the kernel reads (set by its launcher): the y-derivative forms'
    // x and y terms both couple neighbouring components (pattern 1 of
    // XArgs::sopat), qxa = qx[0][1] = qx[1][2], qxb = qx[1][0] = qx[2][1],
    // and likewise qya, qyb; xpat, ypat 0: no such terms
    int xpat, ypat;
    cx<R> qxa, qxb, qya, qyb;
};

constexpr int PSO_WAVES = 8, PSO_RPW = 2;  // wavefronts, rows per wavefront
constexpr int PSO_TX = 64, PSO_TY = PSO_WAVES * PSO_RPW;
static_assert(PSO_WAVES >= 3 && 2 * PSO_TY <= 64, "halo roles: wavefronts 0, 1 and the last; a lane per column point");

template <typename R> struct PsoShared {
    cx<R> yrow[2 * PSO_WAVES + 2][3][PSO_TX];  // 0: the row above the tile; 2w + 1, 2w + 2: the first
                                               // and last row of wavefront w; the last: the row below
    cx<R> xcol[2][PSO_TY][3];                  // the columns left and right of the tile
};

// RENORM scale, CALCNU and HERM of a loaded point (V as in pointwise_kernel).
template <typename R>
__device__ __forceinline__ void pso_pointwise(const SOArgs<R> &a, int x, int y, cx<R> (&v)[3], R d0, R d1, R d2) {
    v[0] = d0 * v[0];
    v[1] = d1 * v[1];
    v[2] = d2 * v[2];
    const R xv = a.x0 + R(x) * a.dx, yv = a.y0 + R(y) * a.dy;
    pointwise(v[0], v[1], v[2], R(0.5) * (xv * xv + a.m.kappa2 * yv * yv), a.m);
}

// FULL: the point is known to lie inside the grid.
template <typename R, bool FULL>
__device__ __forceinline__ void pso_load(const SOArgs<R> &a, int x, int y, cx<R> (&v)[3]) {
    const bool in = FULL || (x >= 0 && x < a.nx && y >= 0 && y < a.ny);
    const long long q = in ? (long long)y * a.nx + x : 0;
#pragma unroll
    for (int j = 0; j < 3; ++j) v[j] = in ? a.src[j * a.plane + q] : czero<R>();
}

// FULL: every tile lies inside the grid (nx and ny multiples of the tile).
template <typename R, bool FULL>
__global__ void __launch_bounds__(64 * PSO_WAVES) __attribute__((amdgpu_waves_per_eu(4))) pso_kernel(SOArgs<R> a) {
    __shared__ PsoShared<R> sh;
    const int lane = threadIdx.x & 63;
    // (w is uniform in the wavefront: the row offsets stay scalar)
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ntx = (a.nx + PSO_TX - 1) / PSO_TX;
    const int x0 = (blockIdx.x % ntx) * PSO_TX, y0 = (blockIdx.x / ntx) * PSO_TY;
    const int x = x0 + lane, yw = y0 + PSO_RPW * w;
    R d0 = R(1), d1 = R(1), d2 = R(1);
    if (a.dscale) {
        d0 = R(a.dscale[0]);
        d1 = R(a.dscale[1]);
        d2 = R(a.dscale[2]);
    }
    // this wavefront's share of the halo first, straight into LDS (zero
    // outside the grid: the pointwise sub-steps keep zero at zero)
    {
        int hx = x, hy = -1;  // the halo point of this lane (hy < 0: none)
        if (w == 0) hy = y0 - 1;
        else if (w == PSO_WAVES - 1) hy = y0 + PSO_TY;
        else if (w == 1 && lane < 2 * PSO_TY) {
            hx = lane < PSO_TY ? x0 - 1 : x0 + PSO_TX;
            hy = y0 + (lane % PSO_TY);
        }
        cx<R> h[3];
        pso_load<R, false>(a, hx, hy, h);
        if (hy >= 0) pso_pointwise(a, hx, hy, h, d0, d1, d2);
        if (w == 0)
#pragma unroll
            for (int j = 0; j < 3; ++j) sh.yrow[0][j][lane] = h[j];
        if (w == PSO_WAVES - 1)
#pragma unroll
            for (int j = 0; j < 3; ++j) sh.yrow[2 * PSO_WAVES + 1][j][lane] = h[j];
        if (w == 1 && lane < 2 * PSO_TY)
#pragma unroll
            for (int j = 0; j < 3; ++j) sh.xcol[lane / PSO_TY][lane % PSO_TY][j] = h[j];
    }
    // the wavefront's rows; the first and last into LDS
    cx<R> v[PSO_RPW][3];
#pragma unroll
    for (int k = 0; k < PSO_RPW; ++k) pso_load<R, FULL>(a, x, yw + k, v[k]);
#pragma unroll
    for (int k = 0; k < PSO_RPW; ++k) pso_pointwise(a, x, yw + k, v[k], d0, d1, d2);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        sh.yrow[2 * w + 1][j][lane] = v[0][j];
        sh.yrow[2 * w + 2][j][lane] = v[PSO_RPW - 1][j];
    }
    __syncthreads();
    // SO update and stores
#pragma unroll
    for (int k = 0; k < PSO_RPW; ++k) {
        cx<R> pv[3], nv[3], dn[3], up[3], u[3];
#pragma unroll
        for (int jp = 0; jp < 3; ++jp) {
            pv[jp] = ror1(v[k][jp]);
            nv[jp] = rol1(v[k][jp]);
            if (lane == 0) pv[jp] = sh.xcol[0][PSO_RPW * w + k][jp];
            if (lane == 63) nv[jp] = sh.xcol[1][PSO_RPW * w + k][jp];
            dn[jp] = k > 0 ? v[k > 0 ? k - 1 : 0][jp] : sh.yrow[2 * w][jp][lane];
            up[jp] = k < PSO_RPW - 1 ? v[k < PSO_RPW - 1 ? k + 1 : 0][jp] : sh.yrow[2 * w + 3][jp][lane];
        }
        // each component's x terms, then its y terms, in the order j' = 0, 1, 2
#pragma unroll
        for (int j = 0; j < 3; ++j) u[j] = v[k][j];
        if (a.xpat) {
            const cx<R> d0 = nv[0] - pv[0], d1 = nv[1] - pv[1], d2 = nv[2] - pv[2];
            u[0] = cfma(a.qxa, d1, u[0]);
            u[1] = cfma(a.qxa, d2, cfma(a.qxb, d0, u[1]));
            u[2] = cfma(a.qxb, d1, u[2]);
        }
        if (a.ypat) {
            const cx<R> d0 = up[0] - dn[0], d1 = up[1] - dn[1], d2 = up[2] - dn[2];
            u[0] = cfma(a.qya, d1, u[0]);
            u[1] = cfma(a.qya, d2, cfma(a.qyb, d0, u[1]));
            u[2] = cfma(a.qyb, d1, u[2]);
        }
        const int y = yw + k;
        if (FULL || (x < a.nx && y < a.ny)) {
            const long long q = (long long)y * a.nx + x;
#pragma unroll
            for (int j = 0; j < 3; ++j) a.dst[j * a.plane + q] = u[j];
        }
    }
}

template <typename R>
__global__ void __launch_bounds__(256) scale_kernel(cx<R> *psi, long long plane, const double *d) {
    const R d0 = R(d[0]), d1 = R(d[1]), d2 = R(d[2]);
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < plane;
         q += (long long)gridDim.x * blockDim.x) {
        psi[q] = d0 * psi[q];
        psi[plane + q] = d1 * psi[plane + q];
        psi[2 * plane + q] = d2 * psi[2 * plane + q];
    }
}

// ---------------------------------------------------------- 1D kernel ---
// A 1D state (3 x nx) fits one workgroup's LDS: the whole run of nsteps
// stays on chip.  Each step is the x-pass above followed, in imaginary time,
// by the norms (exact, within the workgroup) and RENORM, as in the paper.
template <typename R> struct Args1D {
    cx<R> *psi;
    int nx, nsteps;
    R dx, x0;
    Model<R> m;
    LineCoef<R> cx_;
    cx<R> rdiag;
    cx<R> qx[9];
    unsigned qxmask;
    int sopat;                 // what the kernel reads of qx (set by its launcher, so_pattern)
    cx<R> qa, qb;
    RenormSpec sp;
    int renorm;                // 1: the RENORM rule after every step (imaginary
                               // time; real time when asked for)
    double *renorm_out;        // last step's {d, N, fallback}, or nullptr
    // unitary-SO scheme, as in XArgs (line j of the rotated state uses cu[j])
    const cx<R> *ramp;         // [nx], or nullptr
    R rotr[9];
    int rotp[3];
    int rotphased;
    LineCoef<R> cu[3];
    cx<R> rdiag_u[3];
    int strang;                // 1: Strang scheme (with ramp)
};

// USO: the unitary-SO scheme (each wavefront solves its line of the state
// rotated into the SO spin matrix's eigenbasis and phase-symmetrised; the
// state is rotated back in LDS before the RENORM norms).
// The line-solve coefficients are read once into registers (per-lane
// pivots, CM = 0 form): they do not change during the run.
// P2 (with USO): the opt-in Strang scheme, P2(dt/2) before the solve and
// after it (before RENORM), in LDS.
template <typename R, int L, bool USO = false, bool P2 = false>
__global__ void __launch_bounds__(step1d_threads(L)) step1d_kernel(Args1D<R> a) {
    constexpr int NT = step1d_threads(L);
    extern __shared__ unsigned char smem_raw[];
    cx<R> *s = reinterpret_cast<cx<R> *>(smem_raw);
    __shared__ double red[3];
    __shared__ double dsh[8];
    // the step loop's scalars, read from LDS after each barrier instead of
    // being held (and spilled) for the whole run
    struct Consts {
        Model<R> m;
        R x0, dx;
        cx<R> rdiag, qa, qb;
    };
    __shared__ Consts kc;
    if (threadIdx.x == 0) kc = Consts{a.m, a.x0, a.dx, a.rdiag, a.qa, a.qb};
    const int nx = a.nx;
    const int ld = srow<L>(nx);
    const int tid = threadIdx.x;
    const int j = tid >> 6, lane = tid & 63;
    const int start = lane * L;
    const int len = max(0, min(L, nx - start));

    for (int i = tid; i < nx; i += NT) {
        const int si = sidx<L>(i);
        s[si] = a.psi[i];
        s[ld + si] = a.psi[nx + i];
        s[2 * ld + si] = a.psi[2 * nx + i];
    }
    __syncthreads();
    // this lane's elimination coefficients and chunk product, read once for
    // the whole run (the tables do not change between steps)
    const int jc = j < 3 ? j : 0;
    const LineCoef<R> &lc = USO ? a.cu[jc] : a.cx_;
    const ChunkCoef<R, L, 0> ccache(lc, start);
    const cx<R> Acache = lc.chunkA[lane];
    const int lvcache = lc.levels;
    for (int step = 0; step < a.nsteps; ++step) {
        const Model<R> M = kc.m;
        const R kx0 = kc.x0, kdx = kc.dx;
        for (int i = tid; i < nx; i += NT) {
            const int si = sidx<L>(i);
            cx<R> p = s[si], z = s[ld + si], m = s[2 * ld + si];
            const R xv = kx0 + R(i) * kdx;
            if constexpr (P2) {
                Model<R> Mt = M;
                Mt.dt = R(0.5) * M.dt;
                pointwise2(p, z, m, R(0.5) * xv * xv, Mt);
            } else {
                pointwise(p, z, m, R(0.5) * xv * xv, M);
            }
            if constexpr (USO) {
                cx<R> w[3] = {p, z, m};
                uso_in(a, w, a.ramp[i]);
                p = w[0];
                z = w[1];
                m = w[2];
            }
            s[si] = p;
            s[ld + si] = z;
            s[2 * ld + si] = m;
        }
        __syncthreads();
        const bool solver = j < 3;  // wavefront-uniform
        const int jj = solver ? j : 0;
        cx<R> r[L];
        if (solver)
            build_rhs_any<R, L>(jj, s, nullptr, ld, nx, start, len, a.sopat, kc.qa, kc.qb, USO ? a.rdiag_u[jj] : kc.rdiag,
                                r);
        __syncthreads();
        if (solver) solve_line_cached<R, L>(r, len, ccache, Acache, lvcache);
        if constexpr (USO) {
            cx<R> *wj = s + jj * ld;
            if (solver) {
#pragma unroll
                for (int t = 0; t < L; ++t)
                    if (t < len) wj[sidx<L>(start + t)] = uso_ramp_line(jj, a.ramp[start + t]) * r[t];
            }
            __syncthreads();
            for (int i = tid; i < nx; i += NT) {
                const int si = sidx<L>(i);
                cx<R> w[3] = {s[si], s[ld + si], s[2 * ld + si]};
                uso_rotate_out(a, w);
                cx<R> p = w[0], z = w[1], m = w[2];
                if constexpr (P2) {
                    const R xv = a.x0 + R(i) * a.dx;
                    Model<R> Mt = a.m;
                    Mt.dt = R(0.5) * a.m.dt;
                    pointwise2(p, z, m, R(0.5) * xv * xv, Mt);
                }
                s[si] = p;
                s[ld + si] = z;
                s[2 * ld + si] = m;
            }
            __syncthreads();
            if (solver) {
#pragma unroll
                for (int t = 0; t < L; ++t)
                    if (t < len) r[t] = wj[sidx<L>(start + t)];
            }
        }
        if (a.renorm) {
            if (solver) {
                double nrm = 0.0;
#pragma unroll
                for (int t = 0; t < L; ++t)
                    if (t < len) nrm += (double)abs2(r[t]);
#pragma unroll
                for (int d = 32; d >= 1; d >>= 1) nrm += __shfl_down(nrm, d, 64);
                if (lane == 0) red[jj] = nrm;
            }
            __syncthreads();
            if (tid == 0) {
                double N[3] = {red[0] * a.sp.dA, red[1] * a.sp.dA, red[2] * a.sp.dA};
                double d[3], fb = 0.0;
                renorm_factors(a.sp, N, d, &fb);
                for (int q = 0; q < 3; ++q) {
                    dsh[q] = d[q];
                    dsh[3 + q] = N[q];
                }
                dsh[6] = fb;
            }
            __syncthreads();
            if (solver) {
                const R dj = R(dsh[jj]);
#pragma unroll
                for (int t = 0; t < L; ++t)
                    if (t < len) r[t] = dj * r[t];
            }
        }
        if (solver) {
            cx<R> *wj = s + jj * ld;
#pragma unroll
            for (int t = 0; t < L; ++t)
                if (t < len) wj[sidx<L>(start + t)] = r[t];
        }
        __syncthreads();
    }
    for (int i = tid; i < nx; i += NT) {
        const int si = sidx<L>(i);
        a.psi[i] = s[si];
        a.psi[nx + i] = s[ld + si];
        a.psi[2 * nx + i] = s[2 * ld + si];
    }
    if (a.renorm_out && tid < 7 && a.renorm && a.nsteps > 0) a.renorm_out[tid] = dsh[tid];
}

} // namespace ssgp
