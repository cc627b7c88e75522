// step_kernels.hpp -- the SS-CN time step on gfx950.
//
// One step of the spin-1 GP equations (Sec. 3 and App. A of the paper) is
// two device-wide passes over the state:
//   x-pass (one workgroup of 3 wavefronts per row): the renormalisation of
//          the previous imaginary-time step, CALCNU, HERM (pointwise, in the
//          coalesced row layout), then the row of all three components is
//          staged in LDS and each wavefront takes one component: the SO
//          update (x stencil from LDS) builds the Crank-Nicolson right-hand
//          side, and the x line is solved by a chunked Thomas elimination;
//   y-pass (one workgroup per tile of 8 columns and one component): the
//          Crank-Nicolson solve along y, column chunks held in registers, plus
//          the per-tile sums of |psi|^2 for the imaginary-time RENORM.
//
// Chunked Thomas elimination.  The matrix I + sT of every line is the same
// Toeplitz tridiagonal, so the elimination pivots are line independent and
// tabulated on the host: with c'_i the normalised super-diagonal and inv_i
// the reciprocal pivots, the forward sweep is y_i = inv_i r_i - c'_i y_{i-1}
// and the back substitution x_i = y_i - c'_i x_{i+1}.  Each lane owns a
// contiguous chunk of L points.  Both sweeps are first-order linear
// recurrences with the multiplier -c'_i, so a lane first runs its chunk with
// zero carry-in, the chunks are joined by an exact scan of the affine maps
// Y_k = A_k Y_{k-1} + B_k (A_k = prod over the chunk of -c'_i, tabulated),
// and each lane adds the carried term, propagated through the same
// recurrence.  No term is truncated: the result is Thomas elimination up to
// rounding order.
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

// cos(th), sin(th); Taylor series for |th| <= pi/4, library call beyond.
template <typename R> __device__ __forceinline__ void cos_sin(R th, R &c, R &s) {
    const R q = th * th;
    if (q <= SeriesLimit<R>::q) {
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
template <typename R>
__device__ __forceinline__ void pointwise(cx<R> &p, cx<R> &z, cx<R> &m, R V, const Model<R> &M) {
    const R rp = abs2(p), r0 = abs2(z), rm = abs2(m);
    const R rho = rp + r0 + rm;
    const R base = V + M.c0 * rho;
    const R php = base + M.c2 * (rp - rm + r0);
    const R ph0 = base + M.c2 * (rp + rm);
    const R phm = base + M.c2 * (rm - rp + r0);
    if (M.imag) {
        p = exp_(-M.dt * php) * p;
        z = exp_(-M.dt * ph0) * z;
        m = exp_(-M.dt * phm) * m;
    } else {
        R c, s;
        cos_sin(M.dt * php, c, s);
        p = p * mk(c, -s);
        cos_sin(M.dt * ph0, c, s);
        z = z * mk(c, -s);
        cos_sin(M.dt * phm, c, s);
        m = m * mk(c, -s);
    }
    const cx<R> a = cfma(mk(M.c2, R(0)), conj(m) * z, mk(M.om_t, R(0)));
    const cx<R> b = cfma(mk(M.c2, R(0)), conj(z) * p, mk(M.om_t, R(0)));
    const R q = R(0.25) * M.dt * M.dt * (abs2(a) + abs2(b));
    R S, C;
    if (q <= SeriesLimit<R>::q) {
        S = M.imag ? sinhc_q(q) : sinc_q(q);
        C = M.imag ? cosh_q(q) : cos_q(q);
    } else {
        const R u = sqrt_(q);
        if (M.imag) {
            S = sinh_(u) / u;
            C = cosh_(u);
        } else {
            R su, cu;
            sincos_(u, &su, &cu);
            S = su / u;
            C = cu;
        }
    }
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

// -------------------------------------------------- chunked line solve ---
// Forward sweep of one chunk with zero carry-in; r holds the right-hand side
// on entry and the partial y on exit.  Returns the last y (0 if empty).
template <typename R, int L>
__device__ __forceinline__ cx<R> fwd_local(cx<R> (&r)[L], int start, int len,
                                           const cx<R> *__restrict__ inv,
                                           const cx<R> *__restrict__ cp) {
    cx<R> prev = czero<R>();
#pragma unroll
    for (int t = 0; t < L; ++t) {
        if (t < len) {
            const int i = start + t;
            prev = inv[i] * r[t] - cp[i] * prev;
            r[t] = prev;
        }
    }
    return prev;
}

// Adds the carried-in term: e_i = -c'_i e_{i-1}, e_{start-1} = carry.
template <typename R, int L>
__device__ __forceinline__ void fwd_fix(cx<R> (&r)[L], int start, int len,
                                        const cx<R> *__restrict__ cp, cx<R> carry) {
    cx<R> e = carry;
#pragma unroll
    for (int t = 0; t < L; ++t) {
        if (t < len) {
            e = czero<R>() - cp[start + t] * e;
            r[t] = r[t] + e;
        }
    }
}

// Back substitution of one chunk with zero carry-in from the right.
// Returns the first x (0 if empty).
template <typename R, int L>
__device__ __forceinline__ cx<R> bwd_local(cx<R> (&r)[L], int start, int len,
                                           const cx<R> *__restrict__ cp) {
#pragma unroll
    for (int t = L - 2; t >= 0; --t) {
        if (t + 1 < len) r[t] = r[t] - cp[start + t] * r[t + 1];
    }
    return len > 0 ? r[0] : czero<R>();
}

template <typename R, int L>
__device__ __forceinline__ void bwd_fix(cx<R> (&r)[L], int start, int len,
                                        const cx<R> *__restrict__ cp, cx<R> carry) {
    cx<R> e = carry;
#pragma unroll
    for (int t = L - 1; t >= 0; --t) {
        if (t < len) {
            e = czero<R>() - cp[start + t] * e;
            r[t] = r[t] + e;
        }
    }
}

// Inclusive scan over the lanes lane, lane-STRIDE, lane-2*STRIDE, ... of the
// wavefront of the affine maps (A, B): afterwards (A, B) maps the value before
// the first chunk of this wavefront to the value after this lane's chunk.
template <typename R, int STRIDE>
__device__ __forceinline__ void wave_scan_up(cx<R> &A, cx<R> &B) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = STRIDE; d < 64; d <<= 1) {
        const cx<R> Ap = shfl_up(A, d), Bp = shfl_up(B, d);
        if (lane >= d) {
            B = cfma(A, Bp, B);
            A = A * Ap;
        }
    }
}

template <typename R, int STRIDE>
__device__ __forceinline__ void wave_scan_down(cx<R> &A, cx<R> &B) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = STRIDE; d < 64; d <<= 1) {
        const cx<R> Ap = shfl_down(A, d), Bp = shfl_down(B, d);
        if (lane + d < 64) {
            B = cfma(A, Bp, B);
            A = A * Ap;
        }
    }
}

// Solves one line held by the 64 lanes of a wavefront (lane k owns
// [start, start+len)).  Ak = product of -c'_i over the lane's chunk.
template <typename R, int L>
__device__ __forceinline__ void solve_line_wave(cx<R> (&r)[L], int start, int len,
                                                const cx<R> *__restrict__ inv,
                                                const cx<R> *__restrict__ cp, cx<R> Ak) {
    const int lane = threadIdx.x & 63;
    cx<R> A = Ak;
    cx<R> B = fwd_local<R, L>(r, start, len, inv, cp);
    wave_scan_up<R, 1>(A, B);
    cx<R> carry = shfl_up(B, 1);
    if (lane == 0) carry = czero<R>();
    fwd_fix<R, L>(r, start, len, cp, carry);
    A = Ak;
    B = bwd_local<R, L>(r, start, len, cp);
    wave_scan_down<R, 1>(A, B);
    carry = shfl_down(B, 1);
    if (lane == 63) carry = czero<R>();
    bwd_fix<R, L>(r, start, len, cp, carry);
}

// LDS index of point i with one padding slot after every chunk of L points,
// so that the 64 lanes reading "their" chunk hit distinct banks.
template <int L> __device__ __forceinline__ int sidx(int i) { return i + i / L; }
template <int L> __host__ __device__ constexpr int srow(int n) { return n + n / L + 1; }

// ------------------------------------------------------------- x-pass ---
template <typename R> struct XArgs {
    const cx<R> *src;          // state read (3 planes)
    cx<R> *dst;                // state written (may equal src unless so_y)
    int nx, ny;
    long long plane;           // nx * ny
    R dx, dy, x0, y0;
    Model<R> m;
    const double *dscale;      // RENORM factors to apply first, or nullptr
    int pointwise;             // 1: CALCNU + HERM in this pass
    const cx<R> *inv, *cp, *chunkA;  // CN_x tables (nx, nx, 64 entries)
    cx<R> rdiag, roff;         // right-hand side (I - sT): diagonal, off-diagonal
    cx<R> qx[9];               // SO: psi'_j += sum_j' qx[j][j'] (psi_j'(i+1) - psi_j'(i-1))
    unsigned qxmask;           // bit 3j+j' set where qx[j][j'] != 0
    int so_y;                  // 1: add qy terms with rows iy +- 1 of src
    cx<R> qy[9];
    unsigned qymask;
};

constexpr int XPASS_THREADS = 192;

template <typename R, int L>
__global__ void __launch_bounds__(XPASS_THREADS) xpass_kernel(XArgs<R> a) {
    extern __shared__ unsigned char smem_raw[];
    cx<R> *s = reinterpret_cast<cx<R> *>(smem_raw);
    const int nx = a.nx;
    const int ld = srow<L>(nx);
    cx<R> *ys = s + 3 * ld;  // y-derivative SO terms (so_y only)
    const int row = blockIdx.x;
    const int tid = threadIdx.x;
    const long long roff = (long long)row * nx;
    const cx<R> *src = a.src + roff;

    R d0 = R(1), d1 = R(1), d2 = R(1);
    if (a.dscale) {
        d0 = R(a.dscale[0]);
        d1 = R(a.dscale[1]);
        d2 = R(a.dscale[2]);
    }
    const R yv = a.y0 + R(row) * a.dy;
    const R vy = R(0.5) * a.m.kappa2 * yv * yv;
    for (int i = tid; i < nx; i += XPASS_THREADS) {
        cx<R> p = src[i], z = src[a.plane + i], m = src[2 * a.plane + i];
        if (a.dscale) {
            p = d0 * p;
            z = d1 * z;
            m = d2 * m;
        }
        if (a.pointwise) {
            const R xv = a.x0 + R(i) * a.dx;
            pointwise(p, z, m, R(0.5) * xv * xv + vy, a.m);
        }
        const int si = sidx<L>(i);
        s[si] = p;
        s[ld + si] = z;
        s[2 * ld + si] = m;
        if (a.so_y) {
            cx<R> up[3], dn[3];
#pragma unroll
            for (int jp = 0; jp < 3; ++jp) {
                up[jp] = row + 1 < a.ny ? src[jp * a.plane + nx + i] : czero<R>();
                dn[jp] = row >= 1 ? src[jp * a.plane - nx + i] : czero<R>();
            }
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                cx<R> acc = czero<R>();
#pragma unroll
                for (int jp = 0; jp < 3; ++jp)
                    if (a.qymask & (1u << (3 * j + jp))) acc = cfma(a.qy[3 * j + jp], up[jp] - dn[jp], acc);
                ys[j * ld + si] = acc;
            }
        }
    }
    __syncthreads();

    const int j = tid >> 6, lane = tid & 63;
    const int start = lane * L;
    const int len = max(0, min(L, nx - start));
    const cx<R> *sj = s + j * ld;
    // value after the SO sub-step at point i of component j (zero outside)
    auto so_at = [&](int i) -> cx<R> {
        if (i < 0 || i >= nx) return czero<R>();
        cx<R> v = sj[sidx<L>(i)];
        if (a.so_y) v = v + ys[j * ld + sidx<L>(i)];
#pragma unroll
        for (int jp = 0; jp < 3; ++jp) {
            if (a.qxmask & (1u << (3 * j + jp))) {
                const cx<R> fp = i + 1 < nx ? s[jp * ld + sidx<L>(i + 1)] : czero<R>();
                const cx<R> fm = i >= 1 ? s[jp * ld + sidx<L>(i - 1)] : czero<R>();
                v = cfma(a.qx[3 * j + jp], fp - fm, v);
            }
        }
        return v;
    };
    cx<R> r[L];
    cx<R> um = czero<R>(), uc = czero<R>();
    if (len > 0) {
        um = so_at(start - 1);
        uc = so_at(start);
    }
#pragma unroll
    for (int t = 0; t < L; ++t) {
        if (t < len) {
            const cx<R> un = so_at(start + t + 1);
            r[t] = cfma(a.roff, um + un, a.rdiag * uc);
            um = uc;
            uc = un;
        } else {
            r[t] = czero<R>();
        }
    }
    __syncthreads();  // every read of the staged row is done

    solve_line_wave<R, L>(r, start, len, a.inv, a.cp, a.chunkA[lane]);
    cx<R> *wj = s + j * ld;
#pragma unroll
    for (int t = 0; t < L; ++t)
        if (t < len) wj[sidx<L>(start + t)] = r[t];
    __syncthreads();

    cx<R> *dst = a.dst + roff;
    for (int i = tid; i < nx; i += XPASS_THREADS) {
        const int si = sidx<L>(i);
        dst[i] = s[si];
        dst[a.plane + i] = s[ld + si];
        dst[2 * a.plane + i] = s[2 * ld + si];
    }
}

// ------------------------------------------------------------- y-pass ---
template <typename R> struct YArgs {
    cx<R> *psi;                // state, updated in place
    int nx, ny;
    long long plane;
    const cx<R> *inv, *cp, *chunkA;  // CN_y tables (ny, ny, blockDim/TX entries)
    cx<R> rdiag, roff;
    double *norm_partials;     // [3][gridDim.x] sums of |psi|^2, or nullptr
};

constexpr int YPASS_MAX_THREADS = 512;
constexpr int YPASS_MAX_WAVES = YPASS_MAX_THREADS / 64;

// Workgroup: TX adjacent columns x P chunks of L rows (blockDim = TX * P);
// lane tid holds column tid % TX, chunk tid / TX.  grid = (ceil(nx/TX), 3).
template <typename R, int L, int TX>
__global__ void __launch_bounds__(YPASS_MAX_THREADS) ypass_kernel(YArgs<R> a) {
    __shared__ cx<R> scA[2][YPASS_MAX_WAVES][TX], scB[2][YPASS_MAX_WAVES][TX];
    __shared__ double red[YPASS_MAX_WAVES];
    const int nx = a.nx, ny = a.ny;
    const int j = blockIdx.y;
    const int tid = threadIdx.x, c = tid % TX, k = tid / TX;
    const int lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
    const int x = blockIdx.x * TX + c;
    const bool valid = x < nx;
    const int start = k * L;
    const int len = valid ? max(0, min(L, ny - start)) : 0;
    cx<R> *col = a.psi + j * a.plane + (valid ? x : 0);

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
            r[t] = cfma(a.roff, left + right, a.rdiag * f[t]);
        } else {
            r[t] = czero<R>();
        }
    }

    const cx<R> Ak = a.chunkA[k];
    // forward sweep and its scan over the chunks of each column
    cx<R> A = Ak;
    cx<R> B = fwd_local<R, L>(r, start, len, a.inv, a.cp);
    wave_scan_up<R, TX>(A, B);
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
    fwd_fix<R, L>(r, start, len, a.cp, carry);

    // back substitution and its reverse scan
    A = Ak;
    B = bwd_local<R, L>(r, start, len, a.cp);
    wave_scan_down<R, TX>(A, B);
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
    bwd_fix<R, L>(r, start, len, a.cp, carry);

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
            a.norm_partials[(long long)j * gridDim.x + blockIdx.x] = t;
        }
    }
}

// ------------------------------------------------ pointwise-only pass ---
// Used ahead of an x-pass that reads neighbouring rows (y-derivative SO):
// RENORM scale, CALCNU and HERM in place.
template <typename R> struct PArgs {
    cx<R> *psi;
    int nx, ny;
    long long plane;
    R dx, dy, x0, y0;
    Model<R> m;
    const double *dscale;
};

template <typename R>
__global__ void __launch_bounds__(256) pointwise_kernel(PArgs<R> a) {
    const long long n = a.plane;
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
        pointwise(p, z, m, R(0.5) * (xv * xv + a.m.kappa2 * yv * yv), a.m);
        a.psi[q] = p;
        a.psi[n + q] = z;
        a.psi[2 * n + q] = m;
    }
}

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

// Sums the per-tile |psi|^2 partials (fixed order) and writes
// out = {d_+1, d_0, d_-1, N_+1, N_0, N_-1, fallback}.
__global__ void __launch_bounds__(256) renorm_finalize_kernel(const double *partials, int ntiles,
                                                              RenormSpec sp, double *out) {
    __shared__ double red[3][256];
    const int t = threadIdx.x;
    for (int j = 0; j < 3; ++j) {
        double s = 0.0;
        for (int q = t; q < ntiles; q += 256) s += partials[(long long)j * ntiles + q];
        red[j][t] = s;
    }
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (t < w)
            for (int j = 0; j < 3; ++j) red[j][t] += red[j][t + w];
        __syncthreads();
    }
    if (t == 0) {
        double N[3] = {red[0][0] * sp.dA, red[1][0] * sp.dA, red[2][0] * sp.dA};
        double d[3], fb = 0.0;
        renorm_factors(sp, N, d, &fb);
        for (int j = 0; j < 3; ++j) {
            out[j] = d[j];
            out[3 + j] = N[j];
        }
        out[6] = fb;
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
    const cx<R> *inv, *cp, *chunkA;
    cx<R> rdiag, roff;
    cx<R> qx[9];
    unsigned qxmask;
    RenormSpec sp;
    double *renorm_out;        // last step's {d, N, fallback}, or nullptr
};

template <typename R, int L>
__global__ void __launch_bounds__(XPASS_THREADS) step1d_kernel(Args1D<R> a) {
    extern __shared__ unsigned char smem_raw[];
    cx<R> *s = reinterpret_cast<cx<R> *>(smem_raw);
    __shared__ double red[3];
    __shared__ double dsh[8];
    const int nx = a.nx;
    const int ld = srow<L>(nx);
    const int tid = threadIdx.x;
    const int j = tid >> 6, lane = tid & 63;
    const int start = lane * L;
    const int len = max(0, min(L, nx - start));

    for (int i = tid; i < nx; i += XPASS_THREADS) {
        const int si = sidx<L>(i);
        s[si] = a.psi[i];
        s[ld + si] = a.psi[nx + i];
        s[2 * ld + si] = a.psi[2 * nx + i];
    }
    __syncthreads();
    const cx<R> *sj = s + j * ld;
    for (int step = 0; step < a.nsteps; ++step) {
        for (int i = tid; i < nx; i += XPASS_THREADS) {
            const int si = sidx<L>(i);
            cx<R> p = s[si], z = s[ld + si], m = s[2 * ld + si];
            const R xv = a.x0 + R(i) * a.dx;
            pointwise(p, z, m, R(0.5) * xv * xv, a.m);
            s[si] = p;
            s[ld + si] = z;
            s[2 * ld + si] = m;
        }
        __syncthreads();
        auto so_at = [&](int i) -> cx<R> {
            if (i < 0 || i >= nx) return czero<R>();
            cx<R> v = sj[sidx<L>(i)];
#pragma unroll
            for (int jp = 0; jp < 3; ++jp) {
                if (a.qxmask & (1u << (3 * j + jp))) {
                    const cx<R> fp = i + 1 < nx ? s[jp * ld + sidx<L>(i + 1)] : czero<R>();
                    const cx<R> fm = i >= 1 ? s[jp * ld + sidx<L>(i - 1)] : czero<R>();
                    v = cfma(a.qx[3 * j + jp], fp - fm, v);
                }
            }
            return v;
        };
        cx<R> r[L];
        cx<R> um = czero<R>(), uc = czero<R>();
        if (len > 0) {
            um = so_at(start - 1);
            uc = so_at(start);
        }
#pragma unroll
        for (int t = 0; t < L; ++t) {
            if (t < len) {
                const cx<R> un = so_at(start + t + 1);
                r[t] = cfma(a.roff, um + un, a.rdiag * uc);
                um = uc;
                uc = un;
            } else {
                r[t] = czero<R>();
            }
        }
        __syncthreads();
        solve_line_wave<R, L>(r, start, len, a.inv, a.cp, a.chunkA[lane]);
        if (a.m.imag) {
            double nrm = 0.0;
#pragma unroll
            for (int t = 0; t < L; ++t)
                if (t < len) nrm += (double)abs2(r[t]);
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) nrm += __shfl_down(nrm, d, 64);
            if (lane == 0) red[j] = nrm;
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
            const R dj = R(dsh[j]);
#pragma unroll
            for (int t = 0; t < L; ++t)
                if (t < len) r[t] = dj * r[t];
        }
        cx<R> *wj = s + j * ld;
#pragma unroll
        for (int t = 0; t < L; ++t)
            if (t < len) wj[sidx<L>(start + t)] = r[t];
        __syncthreads();
    }
    for (int i = tid; i < nx; i += XPASS_THREADS) {
        const int si = sidx<L>(i);
        a.psi[i] = s[si];
        a.psi[nx + i] = s[ld + si];
        a.psi[2 * nx + i] = s[2 * ld + si];
    }
    if (a.renorm_out && tid < 7 && a.m.imag && a.nsteps > 0) a.renorm_out[tid] = dsh[tid];
}

} // namespace ssgp
