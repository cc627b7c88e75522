// ssgp.hip -- host runtime and C ABI of the MI355X SS-CN stepper
// (declarations and contracts in include/ssgp.h).
//
// A grid owns: the Crank-Nicolson coefficient tables ("COEF" of Table 1 in
// the paper) per axis and propagation mode, the reduction workspace, the
// Omega schedule and the adjoint accumulators.  States stay in the caller's
// buffers.  All work is enqueued on the grid's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/ssgp.h"
#include "launch.hpp"

using namespace ssgp;
using cd = std::complex<double>;

// ------------------------------------------------------------- errors ---
static thread_local std::string g_err;

static int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(SSGP_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));        \
    } while (0)

#define LAUNCH_TRY(expr)                                                                     \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess) return fail(SSGP_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e_)); \
    } while (0)

#define SSGP_TRY(expr)                                                                       \
    do {                                                                                     \
        int rc_ = (expr);                                                                    \
        if (rc_ != SSGP_OK) return rc_;                                                      \
    } while (0)

extern "C" const char *ssgp_last_error(void) { return g_err.c_str(); }
extern "C" const char *ssgp_version(void) { return "ssgp 0.1 (gfx950)"; }

// --------------------------------------------------- device buffers -----
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    int ensure(size_t b) {
        if (b <= bytes) return SSGP_OK;
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        if (hipMalloc(&p, b) != hipSuccess) return fail(SSGP_ENOMEM, "hipMalloc(%zu) failed", b);
        bytes = b;
        return SSGP_OK;
    }
    template <typename T> T *as() const { return static_cast<T *>(p); }
};

// ------------------------------------------------- CN coefficient tables -
// (I + sT) with T = tridiag(-1/(2h^2), 1/h^2, -1/(2h^2)): diagonal
// d = 1 + s/h^2, off-diagonal o = -s/(2h^2).  Thomas pivots m_0 = d,
// m_i = d - o c'_{i-1}, c'_i = o / m_i.  The kernels use y_i = c'_i (r_i/o -
// y_{i-1}), so the right-hand side (I - sT) u is built divided by o.  Chunk
// products A_k = prod_{i in chunk k} (-c'_i) (1 for empty chunks).
struct CNHost {
    std::vector<cd> cp, chunkA;
    cd rdiag;  // (I - sT) / o: diagonal (the off-diagonal is exactly -1)
    int levels;      // scan levels needed for carries above 2^-64
};

// Tables of the symmetric Toeplitz matrix tridiag(o, d, o), with rdiag the
// diagonal of the right-hand-side matrix divided by o (its off-diagonal
// divided by o is -1).
static CNHost cn_tables_do(int n, cd d, cd o, cd rdiag, int L, int nchunks, int max_levels) {
    CNHost t;
    t.cp.resize(n);
    t.cp[0] = o / d;
    for (int i = 1; i < n; ++i) t.cp[i] = o / (d - o * t.cp[i - 1]);
    t.chunkA.assign(nchunks, cd(1.0, 0.0));
    double amax = 0.0;
    for (int k = 0; k < nchunks; ++k) {
        for (int i = k * L; i < std::min(n, (k + 1) * L); ++i) t.chunkA[k] *= -t.cp[i];
        if (k * L < n) amax = std::max(amax, std::abs(t.chunkA[k]));
    }
    t.rdiag = rdiag;
    // A carry from W+1 or more chunks back is scaled by at most amax^(W+1);
    // take the smallest W = 2^levels - 1 with amax^(W+1) <= 2^-64.
    int levels = max_levels;
    if (amax < 1.0) {
        const double need = amax > 0.0 ? 64.0 * std::log(2.0) / -std::log(amax) : 1.0;
        levels = 1;
        while (levels < max_levels && (double)(1 << levels) < need) ++levels;
    }
    t.levels = levels;
    return t;
}

static CNHost cn_tables(int n, double h, cd s, int L, int nchunks, int max_levels) {
    const cd d = 1.0 + s / (h * h), o = -s / (2.0 * h * h);
    return cn_tables_do(n, d, o, (1.0 - s / (h * h)) / o, L, nchunks, max_levels);
}

template <typename R> struct CNDev {
    DevBuf buf;  // cp[n] | chunkA[nchunks] | pw[3 L]
    int n = 0, L = 0, nchunks = 0, head = 1, levels = 6;
    cx<R> rdiag{}, cp_inf{};
    const cx<R> *cp() const { return buf.as<cx<R>>(); }
    const cx<R> *chunkA() const { return buf.as<cx<R>>() + n; }
    const cx<R> *pw() const { return buf.as<cx<R>>() + n + nchunks; }
    LineCoef<R> coef() const {
        LineCoef<R> c;
        c.cp = cp();
        c.chunkA = chunkA();
        c.pw = pw();
        c.cp_inf = cp_inf;
        c.head = head;
        c.levels = levels;
        return c;
    }
};

template <typename R> static cx<R> tor(cd v) { return cx<R>{(R)v.real(), (R)v.imag()}; }
template <typename R> static bool same(cx<R> a, cx<R> b) { return a.x == b.x && a.y == b.y; }

template <typename R>
static int upload_cn(CNDev<R> &dst, const CNHost &h, int n, int L, int nchunks, hipStream_t st) {
    std::vector<cx<R>> host(n + nchunks + 3 * L);
    for (int i = 0; i < n; ++i) host[i] = tor<R>(h.cp[i]);
    for (int k = 0; k < nchunks; ++k) host[n + k] = tor<R>(h.chunkA[k]);
    // the pivots become stationary in the table precision: entries from
    // index head on all equal the last one
    int head = n - 1;
    while (head >= 1 && same(host[head - 1], host[n - 1])) --head;
    // partial products of -c'_i over one chunk, from the pivots as the
    // kernels read them (table precision, stationary beyond head): forward
    // over a chunk of stationary pivots, backward over one, backward over
    // the line's first chunk
    {
        auto piv = [&](int i) {  // entries from head on equal the last
            const cx<R> v = host[std::min(i, n - 1)];
            return cd((double)v.x, (double)v.y);
        };
        const cd tail = piv(n - 1);
        cx<R> *pw = host.data() + n + nchunks;
        cd f(1.0, 0.0), b(1.0, 0.0), b1(1.0, 0.0);
        for (int t = 0; t < L; ++t) {
            f *= -tail;
            pw[t] = tor<R>(f);
        }
        for (int t = L - 1; t >= 0; --t) {
            b *= -tail;
            b1 *= -piv(t);
            pw[L + t] = tor<R>(b);
            pw[2 * L + t] = tor<R>(b1);
        }
    }
    SSGP_TRY(dst.buf.ensure(host.size() * sizeof(cx<R>)));
    HIP_TRY(hipMemcpyAsync(dst.buf.p, host.data(), host.size() * sizeof(cx<R>), hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    dst.n = n;
    dst.L = L;
    dst.nchunks = nchunks;
    dst.head = std::max(head, 1);
    dst.levels = h.levels;
    dst.cp_inf = host[n - 1];
    dst.rdiag = tor<R>(h.rdiag);
    return SSGP_OK;
}

static int pow2_at_least(int v) {
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

// chunk length of an x line handled by one 64-lane wavefront (1D and
// adjoint row kernels, batched x rows)
static int x_chunk(int nx) { return pow2_at_least((nx + 63) / 64); }
// points per thread of the 2D x-pass (256 threads per row)
static int x_block(int nx) { return pow2_at_least((nx + 255) / 256); }

// y-pass shape: TX columns per workgroup, chunks of L rows, P chunks.
// Tiles of 4 columns (64-byte row segments in FP64; the two tiles of a
// 128-byte line run on one XCD) and at most 256 lanes: on MI355X this
// measured faster than 8- or 2-column tiles and than 512-lane tiles (more,
// evenly spread workgroups; e.g. 1024^2: 21.5 us against 26.5 us).
constexpr int YTX = 4;
constexpr int YPASS_LANES = 256;
struct YShape {
    int L, P, threads;
};
static YShape y_shape(int ny) {
    // smallest chunk (8, 16 or 32 rows) with at most 256 lanes per column
    // tile (ny <= 2048 always fits)
    int L = 8;
    while (L < 32 && YTX * ((ny + L - 1) / L) > YPASS_LANES) L <<= 1;
    int P = (ny + L - 1) / L;
    const int per_wave = 64 / YTX;
    P = (P + per_wave - 1) / per_wave * per_wave;
    return {L, P, P * YTX};
}

// ------------------------------------------------------------ SO forms --
// H_SO psi_j = sum_j' hx[j][j'] d_x psi_j' + hy[j][j'] d_y psi_j' (p = -i d).
struct SOForm {
    cd hx[9], hy[9];
};

static void spin_matrices(cd Sx[9], cd Sy[9], cd Sz[9]) {
    const double r = 1.0 / std::sqrt(2.0);
    const cd I(0.0, 1.0);
    const cd sx[9] = {0, r, 0, r, 0, r, 0, r, 0};
    const cd sy[9] = {0, -I * r, 0, I * r, 0, -I * r, 0, I * r, 0};
    const cd sz[9] = {1, 0, 0, 0, 0, 0, 0, 0, -1};
    for (int q = 0; q < 9; ++q) {
        Sx[q] = sx[q];
        Sy[q] = sy[q];
        Sz[q] = sz[q];
    }
}

static SOForm so_form(int so, double gamma) {
    SOForm f;
    for (int q = 0; q < 9; ++q) f.hx[q] = f.hy[q] = 0.0;
    cd Sx[9], Sy[9], Sz[9];
    spin_matrices(Sx, Sy, Sz);
    const cd mi(0.0, -1.0);
    switch (so) {
    case SSGP_SO_PX_SX:
        for (int q = 0; q < 9; ++q) f.hx[q] = mi * gamma * Sx[q];
        break;
    case SSGP_SO_PX_SY:
        for (int q = 0; q < 9; ++q) f.hx[q] = mi * gamma * Sy[q];
        break;
    case SSGP_SO_PX_SZ:
        for (int q = 0; q < 9; ++q) f.hx[q] = mi * gamma * Sz[q];
        break;
    case SSGP_SO_RASHBA:
    case SSGP_SO_DRESSELHAUS:
    case SSGP_SO_ERD: {
        // gamma (eta p_y Sigma_x - p_x Sigma_y)
        const double eta = so == SSGP_SO_RASHBA ? 1.0 : (so == SSGP_SO_DRESSELHAUS ? -1.0 : 0.0);
        for (int q = 0; q < 9; ++q) {
            f.hy[q] = mi * gamma * eta * Sx[q];
            f.hx[q] = -mi * gamma * Sy[q];
        }
        break;
    }
    default:
        break;
    }
    return f;
}

static unsigned nz_mask(const cd *m) {
    unsigned b = 0;
    for (int q = 0; q < 9; ++q)
        if (m[q] != cd(0.0, 0.0)) b |= 1u << q;
    return b;
}

// workgroups of the observables pass (each leaves OBS_NQ partial sums)
constexpr int OBS_MAX_BLOCKS = 1024;  // workgroups of the observables pass (256-point row segments in turn)
static int obs_blocks(int nx, int ny) {
    return (int)std::min<long long>((long long)ny * ((nx + 255) / 256), OBS_MAX_BLOCKS);
}

// --------------------------------------------------------------- grid ---
enum { MODE_REAL = 0, MODE_IMAG = 1, MODE_ADJ = 2, NMODES = 3 };

struct GridCore {
    int dim = 2, nx = 0, ny = 1;
    int ncu = 1;  // compute units of the device
    double dx = 0, dy = 0;
    int dtype = SSGP_C128;
    void *psi = nullptr;
    hipStream_t stream = nullptr;
    ssgp_params p{};
    bool have_params = false;
    std::vector<double> omega_sched;
    int steps_per_seg = 1;
    long long step_index = 0;
    // Omega of the Rabi energy in the observables: params.omega after
    // ssgp_set_params, then the Omega of the last step taken
    double obs_omega = 0.0;
    DevBuf partials, renorm, obs_partials, obs_out, scratch, omega_acc, adj_partials;
    // device-side observables log: OBS_NQ sums per sample
    DevBuf obs_log;
    int obs_log_cap = 0, obs_log_used = 0;
    int built_mode_mask = 0;
    // kernel timing: start/stop events of the x-pass and y-pass kernels of
    // every prof_every-th step (event pairs [x0, x1, y0, y1] per profiled step)
    int prof_every = 0, prof_cap = 0, prof_used = 0;
    long long prof_counter = 0;
    std::vector<hipEvent_t> prof_events;
    // runs of 2D steps replayed as HIP graphs (captured on a private stream,
    // launched on the grid's stream), keyed by everything baked into them
    struct StepGraph {
        int mode, k, renorm_first;
        const void *psi;
        double omega;
        hipGraphExec_t exec;
    };
    std::vector<StepGraph> graphs;
    hipStream_t cap = nullptr;
    int scheme = SSGP_SCHEME_PAPER;
    double uso_wr[9];  // unitary-SO scheme: eigenvectors of the SO spin matrix (columns),
    int uso_p[3];      // as diag(i^uso_p[j]) uso_wr
    bool renorm_real = false;  // RENORM after every real-time step as well
    // steps of this mode end with the RENORM rule
    bool renorms(int mode) const { return mode == MODE_IMAG || (mode == MODE_REAL && renorm_real); }
    void clear_graphs() {
        if (graphs.empty()) return;
        (void)hipStreamSynchronize(stream);  // no replay of them still in flight
        for (StepGraph &x : graphs) (void)hipGraphExecDestroy(x.exec);
        graphs.clear();
    }
    ~GridCore() {
        for (hipEvent_t e : prof_events) (void)hipEventDestroy(e);
        clear_graphs();
        if (cap) (void)hipStreamDestroy(cap);
    }
};

template <typename R> struct Tables {
    CNDev<R> x[NMODES];   // x lines as 64 chunks (1D, adjoint and batched rows)
    CNDev<R> xb[NMODES];  // x lines as 256 chunks (2D x-pass)
    CNDev<R> y[NMODES];
    CNDev<R> xu[NMODES][3];  // unitary-SO scheme: the three symmetrised lines (as x in
    DevBuf ramp[NMODES];     //   1D, as xb in 2D) and the phase ramp of line 0 [nx]
    DevBuf uso_lines[NMODES];  // UsoLines<R> of xu (2D x-pass)
};

struct ssgp_grid_s : GridCore {
    Tables<double> t64;
    Tables<float> t32;
};

static size_t elem_bytes(int dtype) { return dtype == SSGP_C64 ? 8 : 16; }
static double darea(const GridCore &g) { return g.dim == 2 ? g.dx * g.dy : g.dx; }
static long long plane_of(const GridCore &g) { return (long long)g.nx * (g.dim == 2 ? g.ny : 1); }

static cd kfac(int mode) { return mode == MODE_IMAG ? cd(1.0, 0.0) : cd(0.0, 1.0); }
// s = k dt / 2 of the Crank-Nicolson factor; the adjoint of a real-time
// step solves with the conjugate matrices.
static cd cn_s(int mode, double dt) {
    const cd s = 0.5 * kfac(mode) * dt;
    return mode == MODE_ADJ ? std::conj(s) : s;
}

template <typename R> static Tables<R> &tables(ssgp_grid g);
template <> Tables<double> &tables<double>(ssgp_grid g) { return g->t64; }
template <> Tables<float> &tables<float>(ssgp_grid g) { return g->t32; }

// ------------------------------------------------- unitary-SO scheme --
// gamma p_x S_a (a = x, y, z) is solved together with CN_x: the line operator
// is H = T (x) I + (-i d_x) (x) gamma S_a.  With S_a = W diag(1, 0, -1) W^H,
// component c of W^H psi is the scalar line problem (I + sH_c) psi' =
// (I - sH_c) psi, H_c = T + gamma lambda_c (-i d_x): tridiagonal Toeplitz
// with diagonal d = 1 + s/h^2, upper u = s(-1/(2h^2) - i gamma lambda_c/(2h))
// and lower l = s(-1/(2h^2) + i gamma lambda_c/(2h)).  For s = i dt/2 and for
// s = dt/2, |u| = |l|, so rho = sqrt(l/u) has modulus 1, and with
// D = diag(rho^i), D^-1 (I + sH_c) D = tridiag(o, d, o) with o = u rho (and
// the right-hand-side matrix 2I - (I + sH_c) transforms alike).  The line is
// solved as CN_x is, on conj(rho^i) (W^H psi)_c, and multiplied back by rho^i.
// Eigenvectors (columns of W, row-major W[j][c]) of the spin matrix of the
// p_x form, for the eigenvalues 1, 0, -1; the identity without SO.
static void so_eigen(int so, cd W[9], double lam[3], cd S[9]) {
    const double r = 1.0 / std::sqrt(2.0);
    const cd I(0.0, 1.0);
    const cd wx[9] = {0.5, r, 0.5, r, 0.0, -r, 0.5, -r, 0.5};
    const cd wy[9] = {0.5, r, 0.5, I * r, 0.0, -I * r, -0.5, r, -0.5};
    const cd wz[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    cd Sx[9], Sy[9], Sz[9];
    spin_matrices(Sx, Sy, Sz);
    const cd *w = so == SSGP_SO_PX_SX ? wx : so == SSGP_SO_PX_SY ? wy : wz;
    const cd *m = so == SSGP_SO_PX_SX ? Sx : so == SSGP_SO_PX_SY ? Sy : Sz;
    const bool none = so != SSGP_SO_PX_SX && so != SSGP_SO_PX_SY && so != SSGP_SO_PX_SZ;
    for (int q = 0; q < 9; ++q) {
        W[q] = w[q];
        S[q] = none ? cd(0.0) : m[q];
    }
    lam[0] = none ? 0.0 : 1.0;
    lam[1] = 0.0;
    lam[2] = none ? 0.0 : -1.0;
}

// Tables of the three symmetrised lines (chunks of L points, nchunks per
// line) and the phase ramps.
template <typename R> static int build_uso(ssgp_grid g, int mode, int L, int nchunks) {
    Tables<R> &T = tables<R>(g);
    cd W[9], S[9];
    double lam[3];
    // the equal mixture is -gamma p_x Sigma_y
    const bool erd = g->p.so == SSGP_SO_ERD;
    so_eigen(erd ? SSGP_SO_PX_SY : g->p.so, W, lam, S);
    for (int j = 0; j < 3; ++j)  // W diag(lam) W^H must give the spin matrix back
        for (int k = 0; k < 3; ++k) {
            cd m = 0.0;
            for (int c = 0; c < 3; ++c) m += W[3 * j + c] * lam[c] * std::conj(W[3 * k + c]);
            if (std::abs(m - S[3 * j + k]) > 1e-15) return fail(SSGP_EDEVICE, "spin eigenvectors inconsistent");
        }
    // W = diag(i^p_j) Wr with Wr real: the kernels rotate with real numbers
    const cd ipow[4] = {cd(1.0, 0.0), cd(0.0, 1.0), cd(-1.0, 0.0), cd(0.0, -1.0)};
    for (int j = 0; j < 3; ++j) {
        int p = -1;
        for (int k = 0; k < 4 && p < 0; ++k) {
            const cd ph = ipow[k];
            bool ok = true;
            for (int c = 0; c < 3; ++c) ok = ok && std::abs(std::imag(std::conj(ph) * W[3 * j + c])) < 1e-15;
            if (ok) p = k;
        }
        if (p < 0) return fail(SSGP_EDEVICE, "spin eigenvectors: row %d is not a phase times a real row", j);
        g->uso_p[j] = p;
        for (int c = 0; c < 3; ++c) g->uso_wr[3 * j + c] = std::real(std::conj(ipow[p]) * W[3 * j + c]);
    }
    // the eigenvalues are (lambda, 0, -lambda): line 1 has no drift and line
    // 2's ramp is the conjugate of line 0's (the kernels rely on both)
    if (lam[1] != 0.0 || lam[2] != -lam[0]) return fail(SSGP_EDEVICE, "spin eigenvalues not (l, 0, -l)");
    const double h = g->dx, gam = erd ? -g->p.gamma : g->p.gamma;
    const cd s = cn_s(mode, g->p.dt), I(0.0, 1.0);
    const cd d = 1.0 + s / (h * h);
    CNHost tab[3];
    std::vector<cx<R>> ramp((size_t)g->nx);
    int levels = 1;
    cd rho0 = 1.0, o0 = 0.0;
    for (int c = 0; c < 3; ++c) {
        const cd u = s * (-0.5 / (h * h) - I * gam * lam[c] / (2.0 * h));
        cd rho = 1.0;
        if (c == 0) {
            const cd l = s * (-0.5 / (h * h) + I * gam * lam[c] / (2.0 * h));
            rho = std::sqrt(l / u);
            rho /= std::abs(rho);
            rho0 = rho;
        } else if (c == 2) {
            rho = std::conj(rho0);  // sqrt(l/u) of line 2 is the conjugate of line 0's
        }
        const cd o = u * rho;
        if (!(std::abs(d) > 2.0 * std::abs(o)))
            return fail(SSGP_EINVAL, "unitary SO: the line matrix is not diagonally dominant (dt gamma too large)");
        if (c == 2) {
            // o_c^2 = u_c l_c = s^2 (1/(4h^4) + (gamma lambda_c / 2h)^2), and with
            // rho_2 = conj(rho_0), o_2 / o_0 = (l_0 / u_0) (u_0 / l_0) = 1: line 2
            // has line 0's matrix, so it takes line 0's tables (the kernels
            // solve both with one coefficient set)
            if (std::abs(o - o0) > 1e-12 * std::abs(o0)) return fail(SSGP_EDEVICE, "unitary SO: lines 0 and 2 differ");
            tab[2] = tab[0];
            continue;
        }
        if (c == 0) o0 = o;
        tab[c] = cn_tables_do(g->nx, d, o, (2.0 - d) / o, L, nchunks, 6);
        levels = std::max(levels, tab[c].levels);
    }
    const double th = std::arg(rho0);
    for (int i = 0; i < g->nx; ++i) ramp[(size_t)i] = tor<R>(cd(std::cos(th * i), std::sin(th * i)));
    UsoLines<R> ul{};
    for (int c = 0; c < 3; ++c) {
        tab[c].levels = levels;
        SSGP_TRY(upload_cn<R>(T.xu[mode][c], tab[c], g->nx, L, nchunks, g->stream));
        ul.cu[c] = T.xu[mode][c].coef();
        ul.rdiag_u[c] = T.xu[mode][c].rdiag;
    }
    SSGP_TRY(T.uso_lines[mode].ensure(sizeof(UsoLines<R>)));
    HIP_TRY(hipMemcpyAsync(T.uso_lines[mode].p, &ul, sizeof(ul), hipMemcpyHostToDevice, g->stream));
    SSGP_TRY(T.ramp[mode].ensure(ramp.size() * sizeof(cx<R>)));
    HIP_TRY(hipMemcpyAsync(T.ramp[mode].p, ramp.data(), ramp.size() * sizeof(cx<R>), hipMemcpyHostToDevice, g->stream));
    HIP_TRY(hipStreamSynchronize(g->stream));
    return SSGP_OK;
}

template <typename R> static int build_tables(ssgp_grid g, int mode) {
    if (g->built_mode_mask & (1 << mode)) return SSGP_OK;
    g->clear_graphs();  // the graphs hold pointers into the tables
    Tables<R> &T = tables<R>(g);
    const cd s = cn_s(mode, g->p.dt);
    const int Lx = x_chunk(g->nx);
    SSGP_TRY(upload_cn<R>(T.x[mode], cn_tables(g->nx, g->dx, s, Lx, 64, 6), g->nx, Lx, 64, g->stream));
    const bool uso = g->scheme != SSGP_SCHEME_PAPER && mode != MODE_ADJ;  // the joined x solve
    if (g->dim == 1 && uso) SSGP_TRY(build_uso<R>(g, mode, Lx, 64));
    if (g->dim == 2) {
        const int km = x_block(g->nx);
        SSGP_TRY(upload_cn<R>(T.xb[mode], cn_tables(g->nx, g->dx, s, km, XPASS_THREADS, 6), g->nx, km, XPASS_THREADS,
                              g->stream));
        const YShape ys = y_shape(g->ny);
        int maxlv = 0;
        while ((YTX << maxlv) < 64) ++maxlv;
        SSGP_TRY(upload_cn<R>(T.y[mode], cn_tables(g->ny, g->dy, s, ys.L, ys.P, maxlv), g->ny, ys.L, ys.P,
                              g->stream));
        if (uso) SSGP_TRY(build_uso<R>(g, mode, km, XPASS_THREADS));
    }
    g->built_mode_mask |= 1 << mode;
    return SSGP_OK;
}

static bool uses_fixed_m(const ssgp_params &p) {
    if (p.renorm == SSGP_RENORM_NORM) return false;
    if (p.renorm == SSGP_RENORM_FIXED_M) return true;
    const bool commutes = p.so == SSGP_SO_NONE || p.so == SSGP_SO_PX_SZ || p.gamma == 0.0;
    return p.omega == 0.0 && commutes;
}

static bool so_has_y(int so) { return so == SSGP_SO_RASHBA || so == SSGP_SO_DRESSELHAUS || so == SSGP_SO_ERD; }
// y-derivative terms present (the equal mixture, eta = 0, has none: its
// coupling is -gamma p_x Sigma_y alone)
static bool so_y_terms(int so) { return so == SSGP_SO_RASHBA || so == SSGP_SO_DRESSELHAUS; }

static double omega_at(const GridCore &g, long long n) {
    if (g.omega_sched.empty()) return g.p.omega;
    long long s = n / g.steps_per_seg;
    if (s < 0) s = 0;
    if (s >= (long long)g.omega_sched.size()) s = (long long)g.omega_sched.size() - 1;
    return g.omega_sched[(size_t)s];
}

template <typename R> static Model<R> model(const GridCore &g, int mode, double omega) {
    Model<R> m;
    m.c0 = (R)g.p.c0;
    m.c2 = (R)g.p.c2;
    m.dt = (R)g.p.dt;
    m.om_t = (R)(omega / std::sqrt(2.0));
    m.kappa2 = (R)(g.p.kappa * g.p.kappa);
    m.imag = mode == MODE_IMAG ? 1 : 0;
    return m;
}

// ------------------------------------------------------------ launches --
static Launch lc(const GridCore &g) { return Launch{g.stream, g.ncu}; }

template <typename R>
static int launch_x(const GridCore &g, const XArgs<R> &a, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
    Launch c = lc(g);
    c.ev_start = e0;
    c.ev_stop = e1;
    LAUNCH_TRY(launch_xpass<R>(c, a, x_block(g.nx), g.ny));
    return SSGP_OK;
}

template <typename R>
static int launch_y(const GridCore &g, const YArgs<R> &a, const YShape &ys, hipEvent_t e0 = nullptr,
                    hipEvent_t e1 = nullptr) {
    Launch c = lc(g);
    c.ev_start = e0;
    c.ev_stop = e1;
    LAUNCH_TRY(launch_ypass<R>(c, a, ys.L, YTX, ys.threads));
    return SSGP_OK;
}

// SO update psi' = psi - k dt H_SO psi with central differences: the
// coefficients of psi_j'(i+1) - psi_j'(i-1) along x, and along y for the
// argument blocks that carry them (SOArgs).
template <typename R, typename A>
static void fill_so(A &a, const GridCore &g, int mode) {
    const SOForm f = so_form(g.p.so, g.p.gamma);
    const cd k = kfac(mode);
    cd kd = k * g.p.dt;
    if (mode == MODE_ADJ) kd = -kd;  // S^H = I + i dt H in real time
    for (int q = 0; q < 9; ++q) a.qx[q] = tor<R>(-kd * f.hx[q] / (2.0 * g.dx));
    a.qxmask = g.p.so == SSGP_SO_NONE ? 0u : nz_mask(f.hx);
    if constexpr (std::is_same<A, SOArgs<R>>::value) {
        for (int q = 0; q < 9; ++q) a.qy[q] = tor<R>(-kd * f.hy[q] / (2.0 * g.dy));
        a.qymask = g.p.so == SSGP_SO_NONE ? 0u : nz_mask(f.hy);
    }
}

template <typename R>
static XArgs<R> x_args(ssgp_grid g, int mode, const void *src, void *dst, double omega, const double *dscale) {
    Tables<R> &T = tables<R>(g);
    XArgs<R> a{};
    a.src = static_cast<const cx<R> *>(src);
    a.dst = static_cast<cx<R> *>(dst);
    a.nx = g->nx;
    a.ny = g->dim == 2 ? g->ny : 1;
    a.plane = plane_of(*g);
    a.dx = (R)g->dx;
    a.dy = (R)(g->dim == 2 ? g->dy : 0.0);
    a.x0 = (R)(-0.5 * g->nx * g->dx);
    a.y0 = (R)(g->dim == 2 ? -0.5 * g->ny * g->dy : 0.0);
    a.m = model<R>(*g, mode, omega);
    a.dscale = dscale;
    a.pointwise = 1;
    // adjacent rows on one XCD, 16 at a time: at 512 rows the x-pass is 5%
    // faster (and the y-pass after it too); measured no gain at 1024 rows and
    // a loss at 256, where it stays off
    a.rowgrp = (a.ny >= 512 && a.ny < 1024) ? 16 : 0;
    a.cx_ = T.xb[mode].coef();
    a.rdiag = T.x[mode].rdiag;
    fill_so<R>(a, *g, mode);
    a.ramp = nullptr;
    if (g->scheme != SSGP_SCHEME_PAPER && g->dim == 2 && mode != MODE_ADJ) {
        a.strang = g->scheme == SSGP_SCHEME_STRANG ? 1 : 0;
        a.ramp = T.ramp[mode].template as<cx<R>>();
        for (int q = 0; q < 9; ++q) a.rotr[q] = (R)g->uso_wr[q];
        a.rotphased = 0;
        for (int j = 0; j < 3; ++j) {
            a.rotp[j] = g->uso_p[j];
            if (g->uso_p[j] != 0) a.rotphased = 1;
        }
        a.ul = T.uso_lines[mode].template as<UsoLines<R>>();
        a.uso_head = 1;
        for (int c = 0; c < 3; ++c) {
            a.cu[c] = T.xu[mode][c].coef();
            a.rdiag_u[c] = T.xu[mode][c].rdiag;
            a.uso_head = std::max(a.uso_head, a.cu[c].head);
        }
        a.qxmask = 0;  // the SO term is in the line solve
    }
    return a;
}

template <typename R>
static YArgs<R> y_args(ssgp_grid g, int mode, void *psi, double *partials) {
    Tables<R> &T = tables<R>(g);
    YArgs<R> a{};
    a.psi = static_cast<cx<R> *>(psi);
    a.nx = g->nx;
    a.ny = g->ny;
    a.plane = plane_of(*g);
    a.cy = T.y[mode].coef();
    a.rdiag = T.y[mode].rdiag;
    a.norm_partials = partials;
    return a;
}

static RenormSpec renorm_spec(const GridCore &g) {
    RenormSpec sp;
    sp.fixed_m = uses_fixed_m(g.p) ? 1 : 0;
    sp.m = g.p.mag0;
    sp.dA = darea(g);
    return sp;
}

template <typename R> static int adjoint_steps(ssgp_grid g, const void *states, void *lam, int nsteps);

// Workgroups of the element-wise kernels over a plane of n points.
static int ew_blocks(long long n) { return (int)std::min<long long>((n + 255) / 256, 2048); }

// Number of |psi|^2 partials the RENORM of a step reduces: per y-pass tile,
// or (Strang scheme) per workgroup of its closing pointwise pass.
static int renorm_tiles(const GridCore &g) {
    return g.scheme == SSGP_SCHEME_STRANG ? ew_blocks(plane_of(g)) : (g.nx + YTX - 1) / YTX;
}

// Whether a step of this mode continues work left by the step before it:
// the RENORM of the previous step (imaginary time, or real time with
// renorm_real) or, Strang scheme in real time without RENORM, the previous
// step's closing P2(dt/2), merged into this step's x-pass.
static bool uses_cont(const GridCore &g, int mode) {
    return g.renorms(mode) || (g.scheme == SSGP_SCHEME_STRANG && mode == MODE_REAL);
}

// The closing P2(dt/2) of the Strang scheme over psi, in place; with
// partials, the |psi_j|^2 sums of the result per workgroup (for RENORM).
template <typename R>
static int strang_close(ssgp_grid g, int mode, void *psi, double omega, double *partials) {
    PArgs<R> pa{};
    pa.psi = static_cast<cx<R> *>(psi);
    pa.nx = g->nx;
    pa.ny = g->ny;
    pa.plane = plane_of(*g);
    pa.dx = (R)g->dx;
    pa.dy = (R)g->dy;
    pa.x0 = (R)(-0.5 * g->nx * g->dx);
    pa.y0 = (R)(-0.5 * g->ny * g->dy);
    pa.m = model<R>(*g, mode, omega);
    pa.m.dt = (R)(0.5 * g->p.dt);
    pa.dscale = nullptr;
    pa.norm_partials = partials;
    LAUNCH_TRY(launch_pointwise<R>(lc(*g), pa, ew_blocks(pa.plane)));
    return SSGP_OK;
}

// One 2D step from src into dst (dst may equal src except with a
// y-derivative SO form).  cont (see uses_cont): the step continues a run.
// Imaginary time (and real time with renorm_real): with cont the RENORM of
// the previous step (whose last pass left its partials in g->partials) is
// applied first, reduced inside the x-pass; this step leaves its own
// partials.  Strang scheme: the x-pass applies P2(dt/2), twice with cont in
// real time without RENORM (the previous step's closing stage and this
// step's opening one); with RENORM the step closes with its own P2 pass.
template <typename R>
static int step2d(ssgp_grid g, int mode, const void *src, void *dst, double omega, bool cont) {
    const bool rn = g->renorms(mode);
    const bool renorm_prev = cont && rn;
    const bool strang = g->scheme == SSGP_SCHEME_STRANG;
    hipEvent_t *ev = nullptr;
    if (g->prof_every > 0 && (g->prof_counter++ % g->prof_every) == 0 && g->prof_used < g->prof_cap)
        ev = &g->prof_events[(size_t)4 * g->prof_used++];
    const YShape ys = y_shape(g->ny);
    const int rtiles = renorm_tiles(*g);
    if (so_y_terms(g->p.so) && g->p.gamma != 0.0) {
        // RENORM scale, CALCNU, HERM and SO(x, y) from src into scratch, then
        // CN_x from scratch into dst
        const size_t bytes = (size_t)3 * plane_of(*g) * sizeof(cx<R>);
        SSGP_TRY(g->scratch.ensure(bytes));
        if (src == g->scratch.p) return fail(SSGP_EINVAL, "the state is the scratch buffer");
        XArgs<R> xa = x_args<R>(g, mode, g->scratch.p, dst, omega, nullptr);
        SOArgs<R> sa{};
        sa.src = static_cast<const cx<R> *>(src);
        sa.dst = g->scratch.as<cx<R>>();
        sa.nx = g->nx;
        sa.ny = g->ny;
        sa.plane = plane_of(*g);
        sa.dx = (R)g->dx;
        sa.dy = (R)g->dy;
        sa.x0 = (R)(-0.5 * g->nx * g->dx);
        sa.y0 = (R)(-0.5 * g->ny * g->dy);
        sa.m = xa.m;
        sa.dscale = nullptr;
        fill_so<R>(sa, *g, mode);
        if (renorm_prev) {
            LAUNCH_TRY(launch_renorm_finalize(lc(*g), g->partials.as<double>(), rtiles, renorm_spec(*g),
                                              g->renorm.as<double>()));
            sa.dscale = g->renorm.as<double>();
        }
        LAUNCH_TRY(launch_pso<R>(lc(*g), sa));
        xa.pointwise = 0;
        xa.qxmask = 0;  // (the SO update is in the state read)
        SSGP_TRY(launch_x<R>(*g, xa, ev ? ev[0] : nullptr, ev ? ev[1] : nullptr));
    } else {
        XArgs<R> xa = x_args<R>(g, mode, src, dst, omega, nullptr);
        if (renorm_prev) {
            xa.rpart = g->partials.as<double>();
            xa.rntiles = rtiles;
            xa.rsp = renorm_spec(*g);
        }
        if (strang) xa.pointwise = (cont && !rn) ? 2 : 1;
        SSGP_TRY(launch_x<R>(*g, xa, ev ? ev[0] : nullptr, ev ? ev[1] : nullptr));
    }
    YArgs<R> ya = y_args<R>(g, mode, dst, (rn && !strang) ? g->partials.as<double>() : nullptr);
    SSGP_TRY(launch_y<R>(*g, ya, ys, ev ? ev[2] : nullptr, ev ? ev[3] : nullptr));
    if (strang && rn) SSGP_TRY(strang_close<R>(g, mode, dst, omega, g->partials.as<double>()));
    return SSGP_OK;
}

// Longest run of steps replayed as one graph.
constexpr int STEP_GRAPH_MAX = 64;

template <typename R>
static int step_graph(ssgp_grid g, int mode, int k, bool renorm_first, double omega, hipGraphExec_t *out) {
    for (const GridCore::StepGraph &x : g->graphs)
        if (x.mode == mode && x.k == k && x.renorm_first == (int)renorm_first && x.psi == g->psi && x.omega == omega) {
            *out = x.exec;
            return SSGP_OK;
        }
    if (g->graphs.size() >= 32) g->clear_graphs();
    if (!g->cap) HIP_TRY(hipStreamCreateWithFlags(&g->cap, hipStreamNonBlocking));
    // capture on the private stream with kernel timing off
    const hipStream_t saved = g->stream;
    const int saved_every = g->prof_every;
    g->stream = g->cap;
    g->prof_every = 0;
    int rc = SSGP_OK;
    hipError_t e = hipStreamBeginCapture(g->cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        for (int s = 0; s < k && rc == SSGP_OK; ++s)
            rc = step2d<R>(g, mode, g->psi, g->psi, omega, uses_cont(*g, mode) && (renorm_first || s > 0));
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(g->cap, &graph);
        if (e == hipSuccess && rc == SSGP_OK) {
            hipGraphExec_t exec = nullptr;
            e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            if (e == hipSuccess) {
                g->graphs.push_back({mode, k, (int)renorm_first, g->psi, omega, exec});
                *out = exec;
            }
        }
        if (graph) (void)hipGraphDestroy(graph);
    }
    g->stream = saved;
    g->prof_every = saved_every;
    SSGP_TRY(rc);
    if (e != hipSuccess) return fail(SSGP_EDEVICE, "step graph capture failed: %s", hipGetErrorString(e));
    return SSGP_OK;
}

// n in-place 2D steps of g->psi at a fixed Omega.  Runs of steps go out as
// graph replays (runs of 2^i <= 64 steps), except steps whose kernels are
// timed, which are launched one by one.  Every step but the first continues
// the run (uses_cont); the first does when cont_first is set (the RENORM left
// by an earlier call's steps).  Strang scheme in real time without RENORM:
// the run ends with the closing P2(dt/2) of its last step as its own pass.
template <typename R> static int run_steps(ssgp_grid g, int mode, int n, double omega, bool cont_first) {
    if (!g->renorms(mode)) cont_first = false;
    const bool graphable = g->dim == 2;
    // the y-derivative SO forms' pointwise pass writes a scratch copy:
    // allocate it before any capture
    if (so_y_terms(g->p.so) && g->p.gamma != 0.0)
        SSGP_TRY(g->scratch.ensure((size_t)3 * plane_of(*g) * sizeof(cx<R>)));
    int s = 0;
    while (s < n) {
        const bool cont = uses_cont(*g, mode) && (cont_first || s > 0);
        const bool timing = g->prof_every > 0 && g->prof_used < g->prof_cap;
        if (!graphable || (timing && g->prof_counter % g->prof_every == 0)) {
            SSGP_TRY(step2d<R>(g, mode, g->psi, g->psi, omega, cont));
            ++s;
            continue;
        }
        int k = n - s;
        if (timing) k = std::min<long long>(k, g->prof_every - g->prof_counter % g->prof_every);
        int p = 1;
        while (p * 2 <= std::min(k, STEP_GRAPH_MAX)) p *= 2;
        hipGraphExec_t exec = nullptr;
        SSGP_TRY(step_graph<R>(g, mode, p, cont, omega, &exec));
        HIP_TRY(hipGraphLaunch(exec, g->stream));
        if (g->prof_every > 0) g->prof_counter += p;
        s += p;
    }
    if (n > 0 && g->scheme == SSGP_SCHEME_STRANG && !g->renorms(mode))
        SSGP_TRY(strang_close<R>(g, mode, g->psi, omega, nullptr));
    return SSGP_OK;
}

template <typename R> static int launch_1d(ssgp_grid g, int mode, void *psi, int nsteps, double omega) {
    Tables<R> &T = tables<R>(g);
    Args1D<R> a{};
    a.psi = static_cast<cx<R> *>(psi);
    a.nx = g->nx;
    a.nsteps = nsteps;
    a.dx = (R)g->dx;
    a.x0 = (R)(-0.5 * g->nx * g->dx);
    a.m = model<R>(*g, mode, omega);
    a.cx_ = T.x[mode].coef();
    a.rdiag = T.x[mode].rdiag;
    XArgs<R> tmp{};
    fill_so<R>(tmp, *g, mode);
    for (int q = 0; q < 9; ++q) a.qx[q] = tmp.qx[q];
    a.qxmask = tmp.qxmask;
    a.sp = renorm_spec(*g);
    a.renorm_out = g->renorm.as<double>();
    a.renorm = g->renorms(mode) ? 1 : 0;
    a.ramp = nullptr;
    if (g->scheme != SSGP_SCHEME_PAPER && mode != MODE_ADJ) {
        a.strang = g->scheme == SSGP_SCHEME_STRANG ? 1 : 0;
        a.ramp = T.ramp[mode].template as<cx<R>>();
        for (int q = 0; q < 9; ++q) a.rotr[q] = (R)g->uso_wr[q];
        a.rotphased = 0;
        for (int j = 0; j < 3; ++j) {
            a.rotp[j] = g->uso_p[j];
            if (g->uso_p[j] != 0) a.rotphased = 1;
        }
        for (int c = 0; c < 3; ++c) {
            a.cu[c] = T.xu[mode][c].coef();
            a.rdiag_u[c] = T.xu[mode][c].rdiag;
        }
        a.qxmask = 0;  // the SO term is in the line solve
    }
    LAUNCH_TRY(launch_step1d<R>(lc(*g), a, x_chunk(g->nx)));
    return SSGP_OK;
}

// The RENORM of the last 2D step of a call (its last pass left the partials).
template <typename R> static int final_renorm(ssgp_grid g) {
    LAUNCH_TRY(launch_renorm_finalize(lc(*g), g->partials.as<double>(), renorm_tiles(*g), renorm_spec(*g),
                                      g->renorm.as<double>()));
    LAUNCH_TRY(launch_scale<R>(lc(*g), static_cast<cx<R> *>(g->psi), plane_of(*g), g->renorm.as<double>(),
                               ew_blocks(plane_of(*g))));
    return SSGP_OK;
}

template <typename R> static int step_imag_t(ssgp_grid g, int nsteps) {
    SSGP_TRY(build_tables<R>(g, MODE_IMAG));
    if (nsteps > 0) g->obs_omega = g->p.omega;
    if (g->dim == 1) return launch_1d<R>(g, MODE_IMAG, g->psi, nsteps, g->p.omega);
    SSGP_TRY(run_steps<R>(g, MODE_IMAG, nsteps, g->p.omega, false));
    if (nsteps > 0) SSGP_TRY(final_renorm<R>(g));
    return SSGP_OK;
}

template <typename R> static int step_real_t(ssgp_grid g, const void *src, void *dst, int nsteps, bool seq) {
    SSGP_TRY(build_tables<R>(g, MODE_REAL));
    if (nsteps > 0) g->obs_omega = omega_at(*g, g->step_index + nsteps - 1);
    const size_t state_elems = (size_t)3 * plane_of(*g);
    if (g->dim == 1) {
        // 1D: the whole run stays in LDS; split launches where Omega changes
        int done = 0;
        const cx<R> *cur = static_cast<const cx<R> *>(src);
        while (done < nsteps) {
            int chunk = nsteps - done;
            if (!g->omega_sched.empty()) {
                const long long n = g->step_index;
                const long long seg_end = (n / g->steps_per_seg + 1) * g->steps_per_seg;
                chunk = (int)std::min<long long>(chunk, seg_end - n);
            }
            if (seq) chunk = 1;
            cx<R> *out = static_cast<cx<R> *>(dst) + (seq ? (size_t)done * state_elems : 0);
            if (out != cur)
                HIP_TRY(hipMemcpyAsync(out, cur, state_elems * sizeof(cx<R>), hipMemcpyDeviceToDevice, g->stream));
            SSGP_TRY(launch_1d<R>(g, MODE_REAL, out, chunk, omega_at(*g, g->step_index)));
            g->step_index += chunk;
            done += chunk;
            cur = out;
        }
        return SSGP_OK;
    }
    if (!seq && src == g->psi && dst == g->psi) {
        // in place: runs of steps at one Omega
        int done = 0;
        while (done < nsteps) {
            int chunk = nsteps - done;
            if (!g->omega_sched.empty()) {
                const long long n = g->step_index;
                const long long seg_end = (n / g->steps_per_seg + 1) * g->steps_per_seg;
                chunk = (int)std::min<long long>(chunk, seg_end - n);
            }
            // (with renorm_real, a run after the first applies the RENORM
            // that the run before it left)
            SSGP_TRY(run_steps<R>(g, MODE_REAL, chunk, omega_at(*g, g->step_index), done > 0));
            g->step_index += chunk;
            done += chunk;
        }
        if (g->renorm_real && nsteps > 0) SSGP_TRY(final_renorm<R>(g));
        return SSGP_OK;
    }
    const cx<R> *cur = static_cast<const cx<R> *>(src);
    for (int s = 0; s < nsteps; ++s) {
        cx<R> *out = static_cast<cx<R> *>(dst) + (seq ? (size_t)s * state_elems : 0);
        SSGP_TRY(step2d<R>(g, MODE_REAL, cur, out, omega_at(*g, g->step_index), false));
        g->step_index += 1;
        cur = out;
    }
    return SSGP_OK;
}

// ---------------------------------------------------------------- ABI ---
static int check_params(int dim, int scheme, const ssgp_params *p) {
    if (!p) return fail(SSGP_EINVAL, "params is NULL");
    const double v[] = {p->c0, p->c2, p->gamma, p->omega, p->kappa, p->dt, p->mag0};
    for (double x : v)
        if (!std::isfinite(x)) return fail(SSGP_EINVAL, "non-finite parameter");
    if (!(p->dt > 0)) return fail(SSGP_EINVAL, "dt must be > 0 (got %g)", p->dt);
    if (p->so < SSGP_SO_NONE || p->so > SSGP_SO_ERD) return fail(SSGP_EINVAL, "unknown so form %d", p->so);
    if (p->renorm < SSGP_RENORM_AUTO || p->renorm > SSGP_RENORM_FIXED_M)
        return fail(SSGP_EINVAL, "unknown renorm rule %d", p->renorm);
    if (dim == 1 && so_has_y(p->so)) return fail(SSGP_EINVAL, "y-dependent SO form on a 1D grid");
    if (dim == 2 && (p->so == SSGP_SO_PX_SY || p->so == SSGP_SO_PX_SZ))
        return fail(SSGP_EINVAL, "SO form %d is defined for 1D grids", p->so);
    if (std::fabs(p->mag0) > 1.0) return fail(SSGP_EINVAL, "|mag0| must be <= 1");
    if (scheme != SSGP_SCHEME_PAPER && so_y_terms(p->so))
        return fail(SSGP_EINVAL, "the unitary-SO and Strang schemes take the forms without y derivatives");
    return SSGP_OK;
}

static int check_params(const GridCore &g, const ssgp_params *p) { return check_params(g.dim, g.scheme, p); }

extern "C" int ssgp_create_grid(int dim, int nx, int ny, double dx, double dy, int dtype, void *psi_dev,
                                void *hip_stream, ssgp_grid *out) {
    if (!out) return fail(SSGP_EINVAL, "out is NULL");
    *out = nullptr;
    if (dim != 1 && dim != 2) return fail(SSGP_EINVAL, "dim must be 1 or 2");
    if (dtype != SSGP_C128 && dtype != SSGP_C64) return fail(SSGP_EINVAL, "unknown dtype %d", dtype);
    if (dim == 1) ny = 1;
    if (nx < 1 || nx > 2048) return fail(SSGP_EINVAL, "nx must be in [1, 2048] (got %d)", nx);
    if (ny < 1 || ny > 2048) return fail(SSGP_EINVAL, "ny must be in [1, 2048] (got %d)", ny);
    if (!(dx > 0) || !std::isfinite(dx) || (dim == 2 && (!(dy > 0) || !std::isfinite(dy))))
        return fail(SSGP_EINVAL, "grid spacing must be positive");
    if (!psi_dev) return fail(SSGP_EINVAL, "psi_dev is NULL");
    ssgp_grid g = new (std::nothrow) ssgp_grid_s();
    if (!g) return fail(SSGP_ENOMEM, "host allocation failed");
    g->dim = dim;
    g->nx = nx;
    g->ny = ny;
    g->dx = dx;
    g->dy = dim == 2 ? dy : 1.0;
    g->dtype = dtype;
    g->psi = psi_dev;
    g->stream = static_cast<hipStream_t>(hip_stream);
    {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&g->ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || g->ncu < 1) {
            delete g;
            return fail(SSGP_EDEVICE, "cannot query the device");
        }
    }
    // RENORM partials: per y-pass tile, or per workgroup of the Strang
    // scheme's closing pointwise pass
    const int ntiles = std::max((nx + YTX - 1) / YTX, ew_blocks((long long)nx * ny));
    int rc = g->partials.ensure(sizeof(double) * 3 * ntiles);
    if (rc == SSGP_OK) rc = g->renorm.ensure(sizeof(double) * 8);
    if (rc == SSGP_OK) rc = g->obs_partials.ensure(sizeof(double) * OBS_NQ * OBS_MAX_BLOCKS);
    if (rc == SSGP_OK) rc = g->obs_out.ensure(sizeof(double) * 16);
    if (rc == SSGP_OK) rc = g->omega_acc.ensure(sizeof(double) * 1);
    if (rc != SSGP_OK) {
        delete g;
        return rc;
    }
    if (hipMemsetAsync(g->omega_acc.p, 0, sizeof(double), g->stream) != hipSuccess) {
        delete g;
        return fail(SSGP_EDEVICE, "hipMemsetAsync failed");
    }
    *out = g;
    return SSGP_OK;
}

extern "C" int ssgp_set_state(ssgp_grid g, void *psi_dev) {
    if (!g || !psi_dev) return fail(SSGP_EINVAL, "NULL argument");
    g->psi = psi_dev;
    g->clear_graphs();
    return SSGP_OK;
}

extern "C" int ssgp_set_params(ssgp_grid g, const ssgp_params *p) {
    if (!g) return fail(SSGP_EINVAL, "grid is NULL");
    SSGP_TRY(check_params(*g, p));
    if (!g->have_params || p->dt != g->p.dt) g->built_mode_mask = 0;
    g->clear_graphs();  // the graphs hold the model constants
    g->p = *p;
    g->have_params = true;
    g->obs_omega = p->omega;
    return SSGP_OK;
}

extern "C" int ssgp_set_scheme(ssgp_grid g, int scheme) {
    if (!g) return fail(SSGP_EINVAL, "grid is NULL");
    if (scheme != SSGP_SCHEME_PAPER && scheme != SSGP_SCHEME_UNITARY_SO && scheme != SSGP_SCHEME_STRANG)
        return fail(SSGP_EINVAL, "unknown scheme %d", scheme);
    if (scheme != SSGP_SCHEME_PAPER && g->have_params && so_y_terms(g->p.so))
        return fail(SSGP_EINVAL, "the unitary-SO and Strang schemes take the forms without y derivatives");
    if (scheme != g->scheme) {
        g->clear_graphs();
        g->built_mode_mask = 0;
        g->scheme = scheme;
    }
    return SSGP_OK;
}

extern "C" int ssgp_set_renorm_real(ssgp_grid g, int on) {
    if (!g) return fail(SSGP_EINVAL, "grid is NULL");
    if (on != 0 && on != 1) return fail(SSGP_EINVAL, "on must be 0 or 1");
    if ((on != 0) != g->renorm_real) {
        g->clear_graphs();  // the graphs hold the y-pass partials and RENORM reductions or not
        g->renorm_real = on != 0;
    }
    return SSGP_OK;
}

extern "C" int ssgp_set_omega_schedule(ssgp_grid g, const double *omega, int nseg, int steps_per_seg) {
    if (!g) return fail(SSGP_EINVAL, "grid is NULL");
    if (nseg < 0 || (nseg > 0 && (!omega || steps_per_seg < 1))) return fail(SSGP_EINVAL, "bad schedule");
    for (int s = 0; s < nseg; ++s)
        if (!std::isfinite(omega[s])) return fail(SSGP_EINVAL, "non-finite Omega");
    g->omega_sched.assign(omega, omega + nseg);
    g->clear_graphs();
    g->steps_per_seg = nseg > 0 ? steps_per_seg : 1;
    const size_t n = std::max(1, nseg);
    SSGP_TRY(g->omega_acc.ensure(sizeof(double) * n));
    HIP_TRY(hipMemsetAsync(g->omega_acc.p, 0, sizeof(double) * n, g->stream));
    return SSGP_OK;
}

extern "C" int ssgp_set_step_index(ssgp_grid g, long long n) {
    if (!g) return fail(SSGP_EINVAL, "grid is NULL");
    g->step_index = n;
    return SSGP_OK;
}

extern "C" long long ssgp_get_step_index(ssgp_grid g) { return g ? g->step_index : -1; }

extern "C" int ssgp_step_imag(ssgp_grid g, int nsteps) {
    if (!g) return fail(SSGP_EINVAL, "grid is NULL");
    if (!g->have_params) return fail(SSGP_ESTATE, "set_params first");
    if (nsteps < 0) return fail(SSGP_EINVAL, "nsteps < 0");
    return g->dtype == SSGP_C128 ? step_imag_t<double>(g, nsteps) : step_imag_t<float>(g, nsteps);
}

extern "C" int ssgp_step_real(ssgp_grid g, int nsteps) {
    if (!g) return fail(SSGP_EINVAL, "grid is NULL");
    if (!g->have_params) return fail(SSGP_ESTATE, "set_params first");
    if (nsteps < 0) return fail(SSGP_EINVAL, "nsteps < 0");
    return g->dtype == SSGP_C128 ? step_real_t<double>(g, g->psi, g->psi, nsteps, false)
                                 : step_real_t<float>(g, g->psi, g->psi, nsteps, false);
}

extern "C" int ssgp_step_real_seq(ssgp_grid g, const void *src, void *dst, int nsteps) {
    if (!g || !src || !dst) return fail(SSGP_EINVAL, "NULL argument");
    if (!g->have_params) return fail(SSGP_ESTATE, "set_params first");
    if (g->scheme != SSGP_SCHEME_PAPER || g->renorm_real)
        return fail(SSGP_ESTATE, "the adjoint path follows the paper's scheme without real-time RENORM");
    if (nsteps < 0) return fail(SSGP_EINVAL, "nsteps < 0");
    return g->dtype == SSGP_C128 ? step_real_t<double>(g, src, dst, nsteps, true)
                                 : step_real_t<float>(g, src, dst, nsteps, true);
}

// Arguments of the observables pass over psi (Eqs. (4)-(5)) with Rabi
// strength omega.
template <typename R>
static ObsArgs<R> obs_args(int dim, int nx, int ny, double dx, double dy, const ssgp_params &p, double omega,
                           const void *psi) {
    ObsArgs<R> a{};
    a.psi = static_cast<const cx<R> *>(psi);
    a.dim = dim;
    a.nx = nx;
    a.ny = dim == 2 ? ny : 1;
    a.plane = (long long)nx * a.ny;
    a.dx = dx;
    a.dy = dy;
    a.x0 = -0.5 * nx * dx;
    a.y0 = dim == 2 ? -0.5 * ny * dy : 0.0;
    a.kappa2 = p.kappa * p.kappa;
    a.c0 = p.c0;
    a.c2 = p.c2;
    a.om_t = omega / std::sqrt(2.0);
    const SOForm f = so_form(p.so, p.gamma);
    for (int q = 0; q < 9; ++q) {
        a.hx[q] = cx<double>{f.hx[q].real(), f.hx[q].imag()};
        a.hy[q] = cx<double>{f.hy[q].real(), f.hy[q].imag()};
    }
    a.hxmask = p.so == SSGP_SO_NONE ? 0u : nz_mask(f.hx);
    a.hymask = p.so == SSGP_SO_NONE ? 0u : nz_mask(f.hy);
    return a;
}

// Launches the observables pass over psi; the 12 fixed-order sums go to
// out_dev (device memory).  E_rabi takes the Omega of the last step taken
// (GridCore::obs_omega).
template <typename R> static int observables_launch(ssgp_grid g, const void *psi, double *out_dev) {
    ObsArgs<R> a = obs_args<R>(g->dim, g->nx, g->ny, g->dx, g->dy, g->p, g->obs_omega, psi);
    a.partials = g->obs_partials.as<double>();
    const int nb = obs_blocks(a.nx, a.ny);
    LAUNCH_TRY(launch_obs<R>(lc(*g), a, nb));
    LAUNCH_TRY(launch_obs_finalize(lc(*g), g->obs_partials.as<double>(), nb, out_dev));
    return SSGP_OK;
}

// ssgp_obs from the 12 sums of the observables pass (dA the area element).
static int obs_from_sums(double dA, const double *h, ssgp_obs *out) {
    ssgp_obs o{};
    for (int j = 0; j < 3; ++j) o.N[j] = h[j] * dA;
    o.Ntot = o.N[0] + o.N[1] + o.N[2];
    o.M = o.N[0] - o.N[2];
    for (int q = 0; q < 6; ++q) o.E_parts[q] = h[6 + q] * dA;
    o.E = o.E_parts[0] + o.E_parts[1] + o.E_parts[2] + o.E_parts[3] + o.E_parts[4] + o.E_parts[5];
    for (int j = 0; j < 3; ++j) o.rms[j] = h[j] > 0.0 ? std::sqrt(h[3 + j] / h[j]) : 0.0;
    const double nt = h[0] + h[1] + h[2];
    o.rms_tot = nt > 0.0 ? std::sqrt((h[3] + h[4] + h[5]) / nt) : 0.0;
    *out = o;
    if (!std::isfinite(o.Ntot) || !std::isfinite(o.E)) return fail(SSGP_ENONFINITE, "state holds NaN or Inf");
    return SSGP_OK;
}

template <typename R> static int observables_t(ssgp_grid g, const void *psi, ssgp_obs *out) {
    SSGP_TRY(observables_launch<R>(g, psi, g->obs_out.as<double>()));
    double h[OBS_NQ];
    HIP_TRY(hipMemcpyAsync(h, g->obs_out.p, sizeof h, hipMemcpyDeviceToHost, g->stream));
    HIP_TRY(hipStreamSynchronize(g->stream));
    return obs_from_sums(darea(*g), h, out);
}

extern "C" int ssgp_observables(ssgp_grid g, ssgp_obs *out) {
    if (!g || !out) return fail(SSGP_EINVAL, "NULL argument");
    if (!g->have_params) return fail(SSGP_ESTATE, "set_params first");
    return g->dtype == SSGP_C128 ? observables_t<double>(g, g->psi, out) : observables_t<float>(g, g->psi, out);
}

extern "C" int ssgp_obs_log_reserve(ssgp_grid g, int capacity) {
    if (!g) return fail(SSGP_EINVAL, "grid is NULL");
    if (capacity < 0) return fail(SSGP_EINVAL, "capacity < 0");
    HIP_TRY(hipStreamSynchronize(g->stream));  // no record into the old log in flight
    if (capacity > 0) SSGP_TRY(g->obs_log.ensure(sizeof(double) * OBS_NQ * (size_t)capacity));
    g->obs_log_cap = capacity;
    g->obs_log_used = 0;
    return SSGP_OK;
}

extern "C" int ssgp_obs_record(ssgp_grid g) {
    if (!g) return fail(SSGP_EINVAL, "grid is NULL");
    if (!g->have_params) return fail(SSGP_ESTATE, "set_params first");
    if (g->obs_log_used >= g->obs_log_cap) return fail(SSGP_ESTATE, "observables log full (%d samples)", g->obs_log_cap);
    double *slot = g->obs_log.as<double>() + (size_t)OBS_NQ * g->obs_log_used;
    SSGP_TRY(g->dtype == SSGP_C128 ? observables_launch<double>(g, g->psi, slot)
                                   : observables_launch<float>(g, g->psi, slot));
    ++g->obs_log_used;
    return SSGP_OK;
}

extern "C" int ssgp_obs_log_read(ssgp_grid g, ssgp_obs *out, int max, int *count) {
    if (!g || !count || (max > 0 && !out)) return fail(SSGP_EINVAL, "NULL argument");
    if (max < 0) return fail(SSGP_EINVAL, "max < 0");
    const int n = std::min(max, g->obs_log_used);
    std::vector<double> h((size_t)OBS_NQ * std::max(n, 1));
    if (n > 0)
        HIP_TRY(hipMemcpyAsync(h.data(), g->obs_log.p, sizeof(double) * OBS_NQ * n, hipMemcpyDeviceToHost, g->stream));
    HIP_TRY(hipStreamSynchronize(g->stream));
    *count = g->obs_log_used;
    int rc = SSGP_OK;
    for (int k = 0; k < n; ++k) {
        const int r = obs_from_sums(darea(*g), h.data() + (size_t)OBS_NQ * k, out + k);
        if (r != SSGP_OK && rc == SSGP_OK) rc = r;
    }
    return rc;
}

extern "C" int ssgp_step_real_adjoint(ssgp_grid g, const void *states_dev, void *lambda_dev, int nsteps) {
    if (!g || !states_dev || !lambda_dev) return fail(SSGP_EINVAL, "NULL argument");
    if (!g->have_params) return fail(SSGP_ESTATE, "set_params first");
    if (g->scheme != SSGP_SCHEME_PAPER || g->renorm_real)
        return fail(SSGP_ESTATE, "the adjoint path follows the paper's scheme without real-time RENORM");
    if (nsteps < 0) return fail(SSGP_EINVAL, "nsteps < 0");
    return g->dtype == SSGP_C128 ? adjoint_steps<double>(g, states_dev, lambda_dev, nsteps)
                                 : adjoint_steps<float>(g, states_dev, lambda_dev, nsteps);
}

extern "C" int ssgp_omega_grad(ssgp_grid g, double *out, int nseg, int reset) {
    if (!g || !out) return fail(SSGP_EINVAL, "NULL argument");
    const int have = std::max<int>(1, (int)g->omega_sched.size());
    if (nseg != have) return fail(SSGP_EINVAL, "nseg must be %d", have);
    HIP_TRY(hipMemcpyAsync(out, g->omega_acc.p, sizeof(double) * nseg, hipMemcpyDeviceToHost, g->stream));
    HIP_TRY(hipStreamSynchronize(g->stream));
    if (reset) HIP_TRY(hipMemsetAsync(g->omega_acc.p, 0, sizeof(double) * nseg, g->stream));
    return SSGP_OK;
}

extern "C" int ssgp_destroy(ssgp_grid g) {
    if (!g) return SSGP_OK;
    if (g->stream) (void)hipStreamSynchronize(g->stream);
    else (void)hipDeviceSynchronize();
    delete g;
    return SSGP_OK;
}

extern "C" int ssgp_profile(ssgp_grid g, int every, int capacity) {
    if (!g) return fail(SSGP_EINVAL, "grid is NULL");
    if (every < 0 || capacity < 0 || (every > 0 && capacity == 0)) return fail(SSGP_EINVAL, "bad profile request");
    for (hipEvent_t e : g->prof_events) (void)hipEventDestroy(e);
    g->prof_events.clear();
    g->prof_every = 0;
    g->prof_cap = g->prof_used = 0;
    g->prof_counter = 0;
    if (every == 0) return SSGP_OK;
    g->prof_events.resize((size_t)4 * capacity);
    for (auto &e : g->prof_events) HIP_TRY(hipEventCreate(&e));
    g->prof_every = every;
    g->prof_cap = capacity;
    return SSGP_OK;
}

extern "C" int ssgp_profile_read(ssgp_grid g, double *out) {
    if (!g || !out) return fail(SSGP_EINVAL, "NULL argument");
    HIP_TRY(hipStreamSynchronize(g->stream));
    double sx = 0, sy = 0, mx = 1e300, my = 1e300;
    for (int k = 0; k < g->prof_used; ++k) {
        float tx = 0, ty = 0;
        HIP_TRY(hipEventElapsedTime(&tx, g->prof_events[4 * k], g->prof_events[4 * k + 1]));
        HIP_TRY(hipEventElapsedTime(&ty, g->prof_events[4 * k + 2], g->prof_events[4 * k + 3]));
        sx += tx;
        sy += ty;
        mx = std::min(mx, (double)tx);
        my = std::min(my, (double)ty);
    }
    const int n = g->prof_used;
    out[0] = n;
    out[1] = n ? sx / n : 0.0;
    out[2] = n ? sy / n : 0.0;
    out[3] = n ? mx : 0.0;
    out[4] = n ? my : 0.0;
    g->prof_used = 0;
    g->prof_counter = 0;
    return SSGP_OK;
}

#include "adjoint_host.inl"
#include "batch_host.inl"

// ------------------------------------------ observables, no allocation ---
// For callers that cannot allocate device memory: the observables pass's
// partial sums and its result live in this file-scope device array, one copy
// per GPU, held until the process ends.  Host code never passes the array's
// name to a kernel or a copy (on the host it is only a stand-in for the
// symbol): the device address comes from hipGetSymbolAddress, once per
// device, on the first call with that device current.
constexpr int NOALLOC_DOUBLES = OBS_NQ * OBS_MAX_BLOCKS + OBS_NQ;
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

constexpr int NOALLOC_MAX_DEVICES = 64;
static double *g_scratch_ptr[NOALLOC_MAX_DEVICES];
static std::once_flag g_scratch_once[NOALLOC_MAX_DEVICES];
static hipError_t g_scratch_err[NOALLOC_MAX_DEVICES];

static int scratch_on_current_device(double **out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(SSGP_EDEVICE, "device %d beyond the supported %d", dev, NOALLOC_MAX_DEVICES);
    std::call_once(g_scratch_once[dev], [dev]() {
        void *p = nullptr;
        g_scratch_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_scratch_ptr[dev] = static_cast<double *>(p);
    });
    if (g_scratch_err[dev] != hipSuccess || !g_scratch_ptr[dev])
        return fail(SSGP_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(g_scratch_err[dev]));
    *out = g_scratch_ptr[dev];
    return SSGP_OK;
}

template <typename R>
static int observables_noalloc_t(int dim, int nx, int ny, double dx, double dy, const void *psi,
                                 const ssgp_params &p, hipStream_t st, ssgp_obs *out) {
    double *buf = nullptr;
    SSGP_TRY(scratch_on_current_device(&buf));
    ObsArgs<R> a = obs_args<R>(dim, nx, ny, dx, dy, p, p.omega, psi);
    const int nb = obs_blocks(a.nx, a.ny);
    if (nb > OBS_MAX_BLOCKS) return fail(SSGP_EINVAL, "observables need %d partial blocks, scratch holds %d", nb, OBS_MAX_BLOCKS);
    a.partials = buf;                                 // [nb][OBS_NQ], every slot written by its block
    double *sums = buf + OBS_NQ * OBS_MAX_BLOCKS;     // the OBS_NQ final sums
    const Launch c{st, 1};
    LAUNCH_TRY(launch_obs<R>(c, a, nb));
    LAUNCH_TRY(launch_obs_finalize(c, buf, nb, sums));
    double h[OBS_NQ];
    HIP_TRY(hipMemcpyAsync(h, sums, sizeof h, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return obs_from_sums(dim == 2 ? dx * dy : dx, h, out);
}

extern "C" int ssgp_observables_noalloc(int dim, int nx, int ny, double dx, double dy, int dtype,
                                        const void *psi_dev, const ssgp_params *p, void *hip_stream,
                                        ssgp_obs *out) {
    if (!out || !psi_dev) return fail(SSGP_EINVAL, "NULL argument");
    if (dim != 1 && dim != 2) return fail(SSGP_EINVAL, "dim must be 1 or 2");
    if (dtype != SSGP_C128 && dtype != SSGP_C64) return fail(SSGP_EINVAL, "unknown dtype %d", dtype);
    if (dim == 1) ny = 1;
    if (nx < 1 || nx > 2048 || ny < 1 || ny > 2048)
        return fail(SSGP_EINVAL, "nx, ny must be in [1, 2048] (got %d, %d)", nx, ny);
    if (!(dx > 0) || !std::isfinite(dx) || (dim == 2 && (!(dy > 0) || !std::isfinite(dy))))
        return fail(SSGP_EINVAL, "grid spacing must be positive");
    SSGP_TRY(check_params(dim, SSGP_SCHEME_PAPER, p));
    const hipStream_t st = static_cast<hipStream_t>(hip_stream);
    return dtype == SSGP_C128 ? observables_noalloc_t<double>(dim, nx, ny, dx, dim == 2 ? dy : 1.0, psi_dev, *p, st, out)
                              : observables_noalloc_t<float>(dim, nx, ny, dx, dim == 2 ? dy : 1.0, psi_dev, *p, st, out);
}
