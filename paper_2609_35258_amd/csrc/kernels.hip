// HIP kernels of the MLVS-DUGKS step for gfx950.
//
// Work decomposition: one 64-lane wavefront per item (cell, face, ghost row,
// remap); a 256-thread workgroup carries four independent items.  Lanes
// stride over the item's velocity points (velocity index contiguous in
// memory, so every row access is coalesced); velocity-space moments are
// reduced in registers, then across the wave with a fixed butterfly of
// shuffles (deterministic, no LDS and no barriers).  One launch per
// stage covers every level: each item names its own level.  Storage type S is
// float or double; per-velocity arithmetic runs in S; moment sums, the small
// linear solves and the per-cell parameters are double.
#include "mlvs_impl.h"

#include <cmath>
#include <type_traits>

namespace mlvs {

constexpr int BS = 256;             // threads per workgroup
constexpr int WL = 64;              // lanes per wavefront
constexpr int MAXW = BS / WL;       // waves (items) per workgroup
constexpr int RED_MAX = 32;         // largest reduction width

constexpr int NXCD = 8;             // accelerator complex dies (each with its own L2)

__device__ __forceinline__ int lane_id() { return threadIdx.x & (WL - 1); }
// Workgroups are dealt to the XCDs round-robin.  Renumber them so that each
// XCD works through one contiguous range of items: neighbouring faces and
// cells share stencil rows, which then meet in the same L2.  Grids are
// launched as multiples of NXCD, so the renumbering is a bijection.
__device__ __forceinline__ int wg_index() {
    const int per = gridDim.x / NXCD;
    return (blockIdx.x % NXCD) * per + blockIdx.x / NXCD;
}
// The wave index is uniform within a wavefront; readfirstlane tells the
// compiler so, and every per-item quantity then lives in scalar registers.
__device__ __forceinline__ int item0() {
    return __builtin_amdgcn_readfirstlane((int)(wg_index() * MAXW + (threadIdx.x >> 6)));
}
__device__ __forceinline__ int istride() { return gridDim.x * MAXW; }

// A value equal on every lane, moved to scalar registers.
__device__ __forceinline__ double uni(double x) {
    const long long b = __double_as_longlong(x);
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)b);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ float uni(float x) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}

// A double moved across lanes by a DPP pattern (both 32-bit halves).
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ __forceinline__ double read_lane(double x, int lane) {
    const long long b = __double_as_longlong(x);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)b, lane);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Sum NV doubles over the wavefront (all lanes active); every lane receives
// the totals.  Within each row of 16 lanes: DPP exchanges with lane^1, lane^2,
// the mirrored lane of the half row and of the row (each lane then holds its
// row's sum; every step adds two equal-order operands, so all lanes of a row
// agree bit for bit); the four row sums are then combined in a fixed order.
template <int NV>
__device__ __forceinline__ void wave_sum(double (&v)[NV]) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double x = v[k];
        x += dpp_mov<0xB1>(x);     // quad_perm [1,0,3,2]
        x += dpp_mov<0x4E>(x);     // quad_perm [2,3,0,1]
        x += dpp_mov<0x141>(x);    // row_half_mirror
        x += dpp_mov<0x140>(x);    // row_mirror
        v[k] = (read_lane(x, 0) + read_lane(x, 16)) + (read_lane(x, 32) + read_lane(x, 48));
    }
}

// Maximum of NV doubles over the wavefront (all lanes active), same exchanges.
template <int NV>
__device__ __forceinline__ void wave_max(double (&v)[NV]) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double x = v[k];
        x = fmax(x, dpp_mov<0xB1>(x));
        x = fmax(x, dpp_mov<0x4E>(x));
        x = fmax(x, dpp_mov<0x141>(x));
        x = fmax(x, dpp_mov<0x140>(x));
        v[k] = fmax(fmax(read_lane(x, 0), read_lane(x, 16)), fmax(read_lane(x, 32), read_lane(x, 48)));
    }
}

// Device buffers reached through the level descriptors are global memory; the
// address-space cast lets the compiler use global (not flat) loads and stores.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gptr<T> gp(T* p) { return (gptr<T>)p; }

template <typename S>
__device__ __forceinline__ gptr<S> rowp(void* base, size_t off) { return gp(reinterpret_cast<S*>(base)) + off; }

// The velocity of point i as the storage precision's kernels read it: FP64
// storage reads the double coordinates, FP32 storage one (x, y) float pair
// (half the bytes and one load instead of two; the rounding is that of the
// stored values).
template <typename S>
__device__ __forceinline__ void load_xy(const LevelDesc& L, int i, double& x, double& y) {
    if constexpr (sizeof(S) == 4) {
        const unsigned long long b = gp(reinterpret_cast<const unsigned long long*>(L.xy32))[i];
        x = __uint_as_float((unsigned)b);
        y = __uint_as_float((unsigned)(b >> 32));
    } else {
        x = gp(L.xi_x)[i];
        y = gp(L.xi_y)[i];
    }
}

// Gaussian elimination with partial pivoting on a register-resident N x N
// system (all indices compile-time: no scratch).  The pivot search keeps the
// first largest entry, as LAPACK does.  A singular system yields a = 0.
template <int N>
__device__ __forceinline__ void solve_fixed(double (&A)[N][N], double (&b)[N]) {
#pragma unroll
    for (int k = 0; k < N; ++k) {
#pragma unroll
        for (int i = k + 1; i < N; ++i) {
            const bool sw = fabs(A[i][k]) > fabs(A[k][k]);
#pragma unroll
            for (int j = 0; j < N; ++j) {
                const double t = A[k][j];
                A[k][j] = sw ? A[i][j] : t;
                A[i][j] = sw ? t : A[i][j];
            }
            const double t = b[k];
            b[k] = sw ? b[i] : t;
            b[i] = sw ? t : b[i];
        }
#pragma unroll
        for (int i = k + 1; i < N; ++i) {
            const double f = A[k][k] != 0.0 ? A[i][k] / A[k][k] : 0.0;
#pragma unroll
            for (int j = k; j < N; ++j) A[i][j] -= f * A[k][j];
            b[i] -= f * b[k];
        }
    }
#pragma unroll
    for (int k = N - 1; k >= 0; --k) {
        double acc = b[k];
#pragma unroll
        for (int j = k + 1; j < N; ++j) acc -= A[k][j] * b[j];
        b[k] = A[k][k] != 0.0 ? acc / A[k][k] : 0.0;
    }
}

__device__ __forceinline__ double viscosity(double T, const Phys& ph) {
    return ph.mu_ref * pow(T / ph.T_ref, ph.omega);
}

// Macroscopic state from eleven raw moments taken about the shift (u0, v0):
// m = [sum w g, .. x, .. y, .. xx, .. xy, .. yy, .. x|x|^2, .. y|x|^2, sum w h, .. x, .. y]
// (x, y the shifted velocity).  Returns rho, u, v, T and qt = 1/2 sum w c (c^2 g + h).
__device__ __forceinline__ void raw_to_state(const double* m, double u0, double v0, const Phys& ph, double& rho,
                             double& u, double& v, double& T, double& qx, double& qy) {
    rho = m[0];
    const double up = m[1] / rho, vp = m[2] / rho;
    const double E = 0.5 * (m[3] + m[5] + m[8]);
    T = (2.0 * E / rho - (up * up + vp * vp)) / ((3.0 + ph.K) * ph.R);
    const double uu = up * up + vp * vp;
    const double sxx = m[3], syy = m[5], sxy = m[4];
    const double cqx = m[6] - 2.0 * (up * sxx + vp * sxy) + uu * m[1] - up * (sxx + syy)
                       + 2.0 * up * (up * m[1] + vp * m[2]) - up * uu * m[0];
    const double cqy = m[7] - 2.0 * (up * sxy + vp * syy) + uu * m[2] - vp * (sxx + syy)
                       + 2.0 * vp * (up * m[1] + vp * m[2]) - vp * uu * m[0];
    qx = 0.5 * (cqx + m[9] - up * m[8]);
    qy = 0.5 * (cqy + m[10] - vp * m[8]);
    u = u0 + up;
    v = v0 + vp;
}

// Reduced Shakhov target (Eq. g_h_eq_Pr) in evaluation form.  With
// c = xi - u:  g = rn e^{-c^2/2RT} (1 + X.c (c^2/RT - D - 2)),
// h = RT rn e^{-c^2/2RT} (cK + X.c ((c^2/RT - D) cK - 2K)), X = (1-Pr) q/(5 p RT),
// cK = K + 3 - D; the compatibility factor 1 + a . phi (Eq. gh_model_correction)
// with the four-moment basis [1, xi_x, xi_y, E_xi] is folded into b0 + b1 xi_x +
// b2 xi_y + b3 |xi|^2; the eight-moment basis (Eq. eq_eight_basis) adds
// [E_c c_x, E_c c_y, c_x^2 - c_y^2, c_x c_y], E_c = (cK RT + c^2)/2, folded into
// (e4 c_x + e5 c_y)(cK RT + c^2) + e6 (c_x^2 - c_y^2) + e7 c_x c_y.
template <typename C>
struct Eq {
    C rn, ux, uy, i2RT, iRT, RT, Xqx, Xqy;
    C b0, b1, b2, b3;
    C e4, e5, e6, e7, cKRT;
    C cK, Dp2, Dd, K2;
    bool corr, c8;
};

// a: the compatibility coefficients (4, or 8 when ph.compat is 8), or null.
__device__ __forceinline__ Eq<double> make_eq(double rho, double u, double v, double T, double qx, double qy,
                                              const double* a, const Phys& ph) {
    Eq<double> e;
    const double RT = ph.R * T;
    const double D = ph.D;
    e.rn = ph.D == 2 ? rho / (2.0 * M_PI * RT) : rho / sqrt(2.0 * M_PI * RT);
    e.ux = u; e.uy = v;
    e.i2RT = 1.0 / (2.0 * RT);
    e.iRT = 1.0 / RT;
    e.RT = RT;
    const double X = (1.0 - ph.Pr) / (5.0 * rho * RT * RT);
    e.Xqx = X * qx; e.Xqy = X * qy;
    e.cK = ph.K + 3.0 - D;
    e.Dp2 = D + 2.0;
    e.Dd = D;
    e.K2 = 2.0 * ph.K;
    e.corr = (a != nullptr);
    const double Ec0 = 0.5 * (3.0 - D + ph.K) * RT;
    e.b0 = a ? 1.0 + a[0] + a[3] * Ec0 : 1.0;
    e.b1 = a ? a[1] : 0.0;
    e.b2 = a ? a[2] : 0.0;
    e.b3 = a ? 0.5 * a[3] : 0.0;
    e.c8 = a != nullptr && ph.compat == 8;
    e.e4 = e.c8 ? 0.5 * a[4] : 0.0;
    e.e5 = e.c8 ? 0.5 * a[5] : 0.0;
    e.e6 = e.c8 ? a[6] : 0.0;
    e.e7 = e.c8 ? a[7] : 0.0;
    e.cKRT = (3.0 - D + ph.K) * RT;
    return e;
}

// Storage-precision copy held in scalar registers (the values are per item).
template <typename C>
__device__ __forceinline__ Eq<C> eq_cast(const Eq<double>& d) {
    Eq<C> e;
    e.rn = uni((C)d.rn); e.ux = uni((C)d.ux); e.uy = uni((C)d.uy); e.i2RT = uni((C)d.i2RT);
    e.iRT = uni((C)d.iRT); e.RT = uni((C)d.RT); e.Xqx = uni((C)d.Xqx); e.Xqy = uni((C)d.Xqy);
    e.b0 = uni((C)d.b0); e.b1 = uni((C)d.b1); e.b2 = uni((C)d.b2); e.b3 = uni((C)d.b3);
    e.e4 = uni((C)d.e4); e.e5 = uni((C)d.e5); e.e6 = uni((C)d.e6); e.e7 = uni((C)d.e7); e.cKRT = uni((C)d.cKRT);
    e.cK = (C)d.cK; e.Dp2 = (C)d.Dp2; e.Dd = (C)d.Dd; e.K2 = (C)d.K2;
    e.corr = d.corr;
    e.c8 = d.c8;
    return e;
}

// FP32 storage evaluates its Maxwellians with the hardware base-2 exponential
// (two instructions; relative error about 1e-7 |x| in the argument's rounding,
// below the storage precision where the values matter).  The same function
// serves the compatibility sums and every later evaluation of the target, so
// the discrete moments the correction enforces are the ones the step uses.
__device__ __forceinline__ float dexp(float x) { return __expf(x); }
__device__ __forceinline__ double dexp(double x) { return exp(x); }

template <typename C>
__device__ __forceinline__ void eq_eval(const Eq<C>& e, C x, C y, C& g, C& h) {
    const C cx = x - e.ux, cy = y - e.uy;
    const C c2 = cx * cx + cy * cy;
    const C ge = e.rn * dexp(-c2 * e.i2RT);
    const C Xc = cx * e.Xqx + cy * e.Xqy;
    const C c2r = c2 * e.iRT;
    g = ge * (C(1) + Xc * (c2r - e.Dp2));
    h = ge * e.RT * (e.cK + Xc * ((c2r - e.Dd) * e.cK - e.K2));
    if (e.corr) {
        C f = e.b0 + e.b1 * x + e.b2 * y + e.b3 * (x * x + y * y);
        if (e.c8) f += (e.e4 * cx + e.e5 * cy) * (e.cKRT + c2) + e.e6 * (cx * cx - cy * cy) + e.e7 * cx * cy;
        g *= f;
        h *= f;
    }
}

// Velocity points of one item are visited in chunks of U points per lane:
// every load of a chunk is issued before any of its arithmetic, so U loads
// per lane are in flight.  Indices past the end are clamped to the last point
// (a valid address) and their weight is zero.
__device__ __forceinline__ int clampi(int i, int N) { return i < N ? i : N - 1; }

// Compatibility correction (Sec. 3.3.1), part 1: the thirteen velocity sums of
// the uncorrected target over the level that the 4x4 system needs (wave per
// item; every lane receives the totals).
template <typename S, int U>
__device__ __forceinline__ void compat_sums(const LevelDesc& L, const Eq<S>& eu, double (&s)[13]) {
#pragma unroll
    for (int k = 0; k < 13; ++k) s[k] = 0.0;
    const int N = L.N;
    for (int i0 = lane_id(); i0 < N; i0 += WL * U) {
        double xv[U], yv[U], wv[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int i = i0 + q * WL, ic = clampi(i, N);
            xv[q] = gp(L.xi_x)[ic]; yv[q] = gp(L.xi_y)[ic];
            wv[q] = i < N ? gp(L.w)[ic] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const double x = xv[q], y = yv[q];
            S g, h;
            eq_eval<S>(eu, (S)x, (S)y, g, h);
            const double wg = wv[q] * (double)g, wh = wv[q] * (double)h;
            const double x2 = x * x + y * y;
            s[0] += wg; s[1] += wg * x; s[2] += wg * y; s[3] += wg * x * x; s[4] += wg * x * y;
            s[5] += wg * y * y; s[6] += wg * x * x2; s[7] += wg * y * x2; s[8] += wg * x2 * x2;
            s[9] += wh; s[10] += wh * x; s[11] += wh * y; s[12] += wh * x2;
        }
    }
    wave_sum<13>(s);
}

// Part 2 (one lane per item): assemble A and the moment defect from the sums,
// solve, return a[4] (a[2] = 0 in 1-D).
__device__ __forceinline__ void compat_from_sums(const double* s, double rho, double u, double v, double T,
                                                 const Phys& ph, double* a_out) {
    const double E0 = 0.5 * (3.0 - ph.D + ph.K) * ph.R * T;
    const double sx2 = s[3] + s[5];
    const double rhoE = 0.5 * rho * (u * u + v * v) + 0.5 * (3.0 + ph.K) * rho * ph.R * T;
    if (ph.D == 2) {
        double A[4][4] = {{s[0], s[1], s[2], E0 * s[0] + 0.5 * sx2},
                          {s[1], s[3], s[4], E0 * s[1] + 0.5 * s[6]},
                          {s[2], s[4], s[5], E0 * s[2] + 0.5 * s[7]},
                          {0.5 * (sx2 + s[9]), 0.5 * (s[6] + s[10]), 0.5 * (s[7] + s[11]),
                           E0 * 0.5 * (sx2 + s[9]) + 0.5 * (0.5 * s[8] + 0.5 * s[12])}};
        double b[4] = {rho - s[0], rho * u - s[1], rho * v - s[2], rhoE - 0.5 * (sx2 + s[9])};
        solve_fixed<4>(A, b);
        a_out[0] = b[0]; a_out[1] = b[1]; a_out[2] = b[2]; a_out[3] = b[3];
    } else {
        double A[3][3] = {{s[0], s[1], E0 * s[0] + 0.5 * sx2},
                          {s[1], s[3], E0 * s[1] + 0.5 * s[6]},
                          {0.5 * (sx2 + s[9]), 0.5 * (s[6] + s[10]),
                           E0 * 0.5 * (sx2 + s[9]) + 0.5 * (0.5 * s[8] + 0.5 * s[12])}};
        double b[3] = {rho - s[0], rho * u - s[1], rhoE - 0.5 * (sx2 + s[9])};
        solve_fixed<3>(A, b);
        a_out[0] = b[0]; a_out[1] = b[1]; a_out[2] = 0.0; a_out[3] = b[2];
    }
}

// Both parts in one wave (every lane solves the same system).
template <typename S, int U>
__device__ __forceinline__ void compat_solve(const LevelDesc& L, const Eq<S>& eu, double rho, double u, double v,
                                             double T, const Phys& ph, double* a_out) {
    double s[13];
    compat_sums<S, U>(L, eu, s);
    compat_from_sums(s, rho, u, v, T, ph, a_out);
#pragma unroll
    for (int k = 0; k < 4; ++k) a_out[k] = uni(a_out[k]);
}

// Eight-moment compatibility correction (Sec. 3.3.1, Eqs. eq_eight_basis,
// E_c_definition, eq_eight_moment_constraint; D = 2): basis phi = [1, xi_x,
// xi_y, E_xi, E_c c_x, E_c c_y, c_x^2 - c_y^2, c_x c_y], constraint rows
// psi_g = [1, xi_x, xi_y, |xi|^2/2, c^2 c_x/2, c^2 c_y/2, c_x^2 - c_y^2, c_x c_y]
// on g and psi_h = [0, 0, 0, 1/2, c_x/2, c_y/2, 0, 0] on h: mass, momentum,
// energy, the heat flux and a zero deviatoric stress.  Part 1 (wave per item):
// A[k][m] = sum w (psi_g,k g_S + psi_h,k h_S) phi_m, row-major; column 0 holds
// the target's own moments (phi_0 = 1).
template <typename S, int U>
__device__ __forceinline__ void compat_sums8(const LevelDesc& L, const Eq<S>& eu, double u, double v, double T,
                                             const Phys& ph, double (&A)[64]) {
#pragma unroll
    for (int k = 0; k < 64; ++k) A[k] = 0.0;
    const double cKRT = (3.0 - ph.D + ph.K) * ph.R * T;
    const int N = L.N;
    for (int i0 = lane_id(); i0 < N; i0 += WL * U) {
        double xv[U], yv[U], wv[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int i = i0 + q * WL, ic = clampi(i, N);
            xv[q] = gp(L.xi_x)[ic]; yv[q] = gp(L.xi_y)[ic];
            wv[q] = i < N ? gp(L.w)[ic] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const double x = xv[q], y = yv[q];
            S g, h;
            eq_eval<S>(eu, (S)x, (S)y, g, h);
            const double wg = wv[q] * (double)g, wh = wv[q] * (double)h;
            const double cx = x - u, cy = y - v, c2 = cx * cx + cy * cy, x2 = x * x + y * y;
            const double Ec = 0.5 * (cKRT + c2);
            const double phi[8] = {1.0, x, y, 0.5 * (cKRT + x2), Ec * cx, Ec * cy, cx * cx - cy * cy, cx * cy};
            const double kern[8] = {wg, wg * x, wg * y, 0.5 * (wg * x2 + wh), 0.5 * (wg * c2 + wh) * cx,
                                    0.5 * (wg * c2 + wh) * cy, wg * (cx * cx - cy * cy), wg * cx * cy};
#pragma unroll
            for (int k = 0; k < 8; ++k)
#pragma unroll
                for (int mm = 0; mm < 8; ++mm) A[k * 8 + mm] += kern[k] * phi[mm];
        }
    }
    wave_sum<64>(A);
}

// Part 2 (one lane): solve A a = target - A[:, 0] with target [rho, rho u, rho v,
// rho E, q_tar, 0, 0] (q_tar the Shakhov target's own heat flux (1 - Pr) q).
__device__ __forceinline__ void compat_from_sums8(const double* As, double rho, double u, double v, double T,
                                                  double qtx, double qty, const Phys& ph, double* a_out) {
    double A[8][8], b[8];
    for (int k = 0; k < 8; ++k)
        for (int mm = 0; mm < 8; ++mm) A[k][mm] = As[k * 8 + mm];
    const double rhoE = 0.5 * rho * (u * u + v * v) + 0.5 * (3.0 + ph.K) * rho * ph.R * T;
    const double tgt[8] = {rho, rho * u, rho * v, rhoE, qtx, qty, 0.0, 0.0};
    for (int k = 0; k < 8; ++k) b[k] = tgt[k] - As[k * 8];
    solve_fixed<8>(A, b);
    for (int k = 0; k < 8; ++k) a_out[k] = b[k];
}

// The correction in one wave for the compatibility order of ph (4 or 8
// moments; every lane solves the same system).  qx, qy: the target's q.
template <typename S, int U>
__device__ __forceinline__ void compat_solve_any(const LevelDesc& L, const Eq<S>& eu, double rho, double u, double v,
                                                 double T, double qx, double qy, const Phys& ph, double* a_out) {
    if (ph.compat == 8) {
        double A[64];
        compat_sums8<S, U>(L, eu, u, v, T, ph, A);
        compat_from_sums8(A, rho, u, v, T, (1.0 - ph.Pr) * qx, (1.0 - ph.Pr) * qy, ph, a_out);
#pragma unroll
        for (int k = 0; k < 8; ++k) a_out[k] = uni(a_out[k]);
    } else {
        compat_solve<S, U>(L, eu, rho, u, v, T, ph, a_out);
    }
}

// Eleven raw moments of (g, h) at velocity (x, y) taken about a shift (the
// layout raw_to_state reads), accumulated in double.
template <typename S>
__device__ __forceinline__ void acc_raw(double* m, double w, double x, double y, S g, S h) {
    const double wg = w * (double)g, wh = w * (double)h;
    const double x2 = x * x + y * y;
    m[0] += wg; m[1] += wg * x; m[2] += wg * y; m[3] += wg * x * x; m[4] += wg * x * y;
    m[5] += wg * y * y; m[6] += wg * x * x2; m[7] += wg * y * x2;
    m[8] += wh; m[9] += wh * x; m[10] += wh * y;
}

// ---------------------------------------------------------------------------
// Staged kernels.  A workgroup of GWV waves takes GW = GWV x IPW items.
// Velocity passes run with one wave per item (lanes over the item's points,
// IPW items per wave in turn); the per-item scalar steps (state, relaxation
// time, the small solves) run once per item on one lane of wave 0, and the two
// kinds of step hand their results over through LDS.  The scalar work is not
// repeated on 64 lanes.
// ---------------------------------------------------------------------------
#ifndef MLVS_STAGED_IPW
#define MLVS_STAGED_IPW 1
#endif
constexpr int GWV = 8;
constexpr int IPW = MLVS_STAGED_IPW;
constexpr int GW = GWV * IPW;
constexpr int GBS = GWV * WL;
static_assert(GW <= WL, "the scalar steps of a workgroup run on the lanes of one wave");

// Velocity chunks.  Streaming stages that reuse neighbours' rows (face
// reconstruction, update) split each item's points into chunks of CH points
// and take (chunk, item) pairs chunk-major, so the waves resident on an XCD
// work on the same velocity range of neighbouring items and their rows meet in
// that XCD's L2.  Each pair writes partial sums; the next stage adds the
// chunks of an item in chunk order (fixed order: deterministic).
__device__ __forceinline__ void sum_chunks(const double* part, int item, int n_items, int N, int CH, double* out) {
    const int nch = (N + CH - 1) / CH;
    for (int j = 0; j < 11; ++j) out[j] = 0.0;
    for (int k = 0; k < nch; ++k) {
        const double* q = part + ((size_t)k * n_items + item) * NMOM;
        for (int j = 0; j < 11; ++j) out[j] += q[j];
    }
    out[M_U0] = part[(size_t)item * NMOM + M_U0];
    out[M_V0] = part[(size_t)item * NMOM + M_V0];
}

// Cell state from the raw moments (Eqs. W_from_tilde, discrete_q): W, tau,
// q = 2 tau q~/(2 tau + dt Pr), and the update weights
// alpha = (2 tau - s)/(2 tau + dt), beta = 3 s/(2 tau + dt), s = dt/2.
struct CellState { double rho, u, v, T, qx, qy, tau, alpha, beta; };

__device__ __forceinline__ CellState cell_state(const double* cm, const Phys& ph) {
    double m[11];
#pragma unroll
    for (int k = 0; k < 11; ++k) m[k] = cm[k];
    CellState c;
    raw_to_state(m, cm[M_U0], cm[M_V0], ph, c.rho, c.u, c.v, c.T, c.qx, c.qy);
    const double p = c.rho * ph.R * c.T;
    c.tau = viscosity(c.T, ph) / p;
    const double dt = ph.dt, s = 0.5 * dt;
    c.qx = 2.0 * c.tau * c.qx / (2.0 * c.tau + dt * ph.Pr);
    c.qy = 2.0 * c.tau * c.qy / (2.0 * c.tau + dt * ph.Pr);
    c.alpha = (2.0 * c.tau - s) / (2.0 * c.tau + dt);
    c.beta = 3.0 * s / (2.0 * c.tau + dt);
    return c;
}

// Cell stage: W, q, tau, compatibility coefficients (written to params) and
// the rows phi_bar+ = alpha phi~ + beta phi_S* (Eq. g_h_eq_Pr with the
// correction of Sec. 3.3.1).  The raw moments of g~, h~ come from cmom (the
// previous update, or k_raw_moments after the state was set from outside).
// The phi_bar+ row of one cell (Eq. bar_phi_transport): phi_bar+ = alpha
// phi~ + beta phi_S* at every point of its level, phi_S* the (corrected)
// target e.
template <typename S, int U>
__device__ __forceinline__ void phibar_points(const LevelDesc& L, size_t row, const Eq<double>& ed, double alpha,
                                              double beta) {
    const int N = L.N;
    auto g = rowp<S>(L.g, row);
    auto h = rowp<S>(L.h, row);
    auto fg = rowp<S>(L.fg, row);
    auto fh = rowp<S>(L.fh, row);
    const Eq<S> e = eq_cast<S>(ed);
    const S al = uni((S)alpha), be = uni((S)beta);
    for (int i0 = lane_id(); i0 < N; i0 += WL * U) {
        S gv[U], hv[U], xv[U], yv[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int ic = clampi(i0 + q * WL, N);
            gv[q] = g[ic]; hv[q] = h[ic];
            double xd, yd;
            load_xy<S>(L, ic, xd, yd);
            xv[q] = (S)xd; yv[q] = (S)yd;
        }
#pragma unroll
        for (int q = 0; q < U; ++q) {
            S gs, hs;
            eq_eval<S>(e, xv[q], yv[q], gs, hs);
            gv[q] = al * gv[q] + be * gs;
            hv[q] = al * hv[q] + be * hs;
        }
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int i = i0 + q * WL;
            if (i < N) { fg[i] = gv[q]; fh[i] = hv[q]; }
        }
    }
}

// The corrected cell target in one wave (every lane holds the result): the
// compatibility sums over the level's points and the small solve (four or
// eight moments), for a cell whose state and uncorrected target are given.
template <typename S, int U, int CM>
__device__ __forceinline__ void cell_target_wave(const LevelDesc& L, const CellState& cs, const Phys& ph,
                                                 Eq<double>& e, double (&a)[8]) {
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = 0.0;
    if (!ph.compat) return;
    if constexpr (CM == 8) {
        double A[64];
        compat_sums8<S, U>(L, eq_cast<S>(e), cs.u, cs.v, cs.T, ph, A);
        compat_from_sums8(A, cs.rho, cs.u, cs.v, cs.T, (1.0 - ph.Pr) * cs.qx, (1.0 - ph.Pr) * cs.qy, ph, a);
    } else {
        double sm[13];
        compat_sums<S, U>(L, eq_cast<S>(e), sm);
        compat_from_sums(sm, cs.rho, cs.u, cs.v, cs.T, ph, a);
    }
    e = make_eq(cs.rho, cs.u, cs.v, cs.T, cs.qx, cs.qy, a, ph);
}

__device__ __forceinline__ void write_params(double* pr, const CellState& cs, const double* a) {
    pr[P_RHO] = cs.rho; pr[P_U] = cs.u; pr[P_V] = cs.v; pr[P_T] = cs.T; pr[P_QX] = cs.qx;
    pr[P_QY] = cs.qy; pr[P_TAU] = cs.tau; pr[P_A0] = a[0]; pr[P_A1] = a[1]; pr[P_A2] = a[2];
    pr[P_A3] = a[3]; pr[P_ALPHA] = cs.alpha; pr[P_BETA] = cs.beta;
}

template <typename S, int U, int MINW, int CM>
__global__ __launch_bounds__(GBS, MINW) void k_cell_prep(const LevelDesc* __restrict__ lvs,
                                                         const int* __restrict__ cell_lev,
                                                         const int* __restrict__ cell_slot,
                                                         const int* __restrict__ order, int n_cells, Phys ph,
                                                         double* __restrict__ params,
                                                         const double* __restrict__ cmom, int CH) {
    constexpr int NS = CM == 8 ? 64 : 13;      // compatibility sums per item
    __shared__ CellState sh_c[GW];
    __shared__ Eq<double> sh_e[GW];
    __shared__ double sh_s[GW][NS];
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));   // wave index (uniform)
    const int t = threadIdx.x;
    for (int g0 = wg_index() * GW; g0 < n_cells; g0 += gridDim.x * GW) {
        // scalar: state and the uncorrected target, one lane per cell
        if (t < GW && g0 + t < n_cells) {
            const int ci = order[g0 + t];
            double cm[NMOM];
            sum_chunks(cmom, ci, n_cells, lvs[cell_lev[ci]].N, CH, cm);
            const CellState cs = cell_state(cm, ph);
            sh_c[t] = cs;
            sh_e[t] = make_eq(cs.rho, cs.u, cs.v, cs.T, cs.qx, cs.qy, nullptr, ph);
        }
        __syncthreads();
        // velocity pass: the compatibility sums, one wave per cell
        for (int kk = 0; kk < IPW; ++kk) {
            const int j = w + GWV * kk;
            const int c = g0 + j < n_cells ? order[g0 + j] : n_cells;
            if (ph.compat && c < n_cells) {
                const LevelDesc& L = lvs[cell_lev[c]];
                double sm[NS];
                if constexpr (CM == 8) {
                    const CellState& cs = sh_c[j];
                    compat_sums8<S, U>(L, eq_cast<S>(sh_e[j]), cs.u, cs.v, cs.T, ph, sm);
                } else {
                    compat_sums<S, U>(L, eq_cast<S>(sh_e[j]), sm);
                }
                if (lane_id() < NS) {
#pragma unroll
                    for (int k = 0; k < NS; ++k)
                        if (lane_id() == k) sh_s[j][k] = sm[k];
                }
            }
        }
        __syncthreads();
        // scalar: solve, corrected target, parameters
        if (t < GW && g0 + t < n_cells) {
            const CellState cs = sh_c[t];
            double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            if (ph.compat) {
                if constexpr (CM == 8)
                    compat_from_sums8(sh_s[t], cs.rho, cs.u, cs.v, cs.T, (1.0 - ph.Pr) * cs.qx,
                                      (1.0 - ph.Pr) * cs.qy, ph, a);
                else
                    compat_from_sums(sh_s[t], cs.rho, cs.u, cs.v, cs.T, ph, a);
                sh_e[t] = make_eq(cs.rho, cs.u, cs.v, cs.T, cs.qx, cs.qy, a, ph);
            }
            write_params(params + (size_t)order[g0 + t] * NPARAM, cs, a);
        }
        __syncthreads();
        // velocity pass: the phi_bar+ rows
        for (int kk = 0; kk < IPW; ++kk) {
            const int j = w + GWV * kk;
            const int c = g0 + j < n_cells ? order[g0 + j] : n_cells;
            if (c >= n_cells) break;
            const LevelDesc& L = lvs[cell_lev[c]];
            phibar_points<S, U>(L, (size_t)cell_slot[c] * L.stride, sh_e[j], sh_c[j].alpha, sh_c[j].beta);
        }
        __syncthreads();
    }
}

// Raw moments of the stored g~, h~ about the cell velocity held in params (used
// when the state was written by anything other than the update), per (chunk,
// cell) pair in the layout the update writes.
template <typename S>
__global__ __launch_bounds__(BS) void k_raw_moments(const LevelDesc* __restrict__ lvs, const int* __restrict__ cell_lev,
                                                    const int* __restrict__ cell_slot, int n_cells,
                                                    const double* __restrict__ params, double* __restrict__ cmom,
                                                    int CH, int nch) {
    constexpr int U = 4;
    const int n = n_cells * nch;
    for (int it = item0(); it < n; it += istride()) {
        const int k = it / n_cells, c = it - k * n_cells;
        const LevelDesc& L = lvs[cell_lev[c]];
        const int beg = k * CH;
        if (beg >= L.N) continue;
        const int end = min(L.N, beg + CH);
        const size_t row = (size_t)cell_slot[c] * L.stride;
        auto g = rowp<S>(L.g, row);
        auto h = rowp<S>(L.h, row);
        const double u0 = params[(size_t)c * NPARAM + P_U], v0 = params[(size_t)c * NPARAM + P_V];
        double m[11];
#pragma unroll
        for (int j = 0; j < 11; ++j) m[j] = 0.0;
        for (int i0 = beg + lane_id(); i0 < end; i0 += WL * U) {
            S gv[U], hv[U];
            double xv[U], yv[U], wv[U];
#pragma unroll
            for (int q = 0; q < U; ++q) {
                const int i = i0 + q * WL, ic = clampi(i, end);
                gv[q] = g[ic]; hv[q] = h[ic];
                xv[q] = gp(L.xi_x)[ic]; yv[q] = gp(L.xi_y)[ic];
                wv[q] = i < end ? gp(L.w)[ic] : 0.0;
            }
#pragma unroll
            for (int q = 0; q < U; ++q) acc_raw<S>(m, wv[q], xv[q] - u0, yv[q] - v0, gv[q], hv[q]);
        }
        wave_sum<11>(m);
        if (lane_id() == 0) {
            double* o = cmom + (size_t)it * NMOM;
            for (int j = 0; j < 11; ++j) o[j] = m[j];
            o[M_U0] = u0;
            o[M_V0] = v0;
        }
    }
}

// Equilibrium start: g~ = g_eq*, h~ = h_eq* at (rho, u, v, T), q = 0.
template <typename S>
__global__ __launch_bounds__(BS) void k_init_eq(const LevelDesc* __restrict__ lvs, const int* __restrict__ cell_lev,
                                                const int* __restrict__ cell_slot, int n_cells,
                                                const double* __restrict__ st, Phys ph, double* __restrict__ params) {
    for (int c = item0(); c < n_cells; c += istride()) {
        const LevelDesc& L = lvs[cell_lev[c]];
        const double rho = st[4 * c], u = st[4 * c + 1], v = ph.D == 2 ? st[4 * c + 2] : 0.0, T = st[4 * c + 3];
        double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        if (ph.compat) {
            const Eq<S> eu = eq_cast<S>(make_eq(rho, u, v, T, 0.0, 0.0, nullptr, ph));
            compat_solve_any<S, 4>(L, eu, rho, u, v, T, 0.0, 0.0, ph, a);
        }
        const Eq<S> e = eq_cast<S>(make_eq(rho, u, v, T, 0.0, 0.0, ph.compat ? a : nullptr, ph));
        const size_t row = (size_t)cell_slot[c] * L.stride;
        auto g = rowp<S>(L.g, row);
        auto h = rowp<S>(L.h, row);
        for (int i = lane_id(); i < L.N; i += WL) {
            S gs, hs;
            eq_eval<S>(e, (S)gp(L.xi_x)[i], (S)gp(L.xi_y)[i], gs, hs);
            g[i] = gs;
            h[i] = hs;
        }
        if (lane_id() == 0) {
            double* pr = params + (size_t)c * NPARAM;
            for (int k = 0; k < NPARAM; ++k) pr[k] = 0.0;
            pr[P_RHO] = rho; pr[P_U] = u; pr[P_V] = v; pr[P_T] = T;
        }
    }
}

// ---------------------------------------------------------------------------
// neighbours on other levels: projection + linear mapping correction
// ---------------------------------------------------------------------------
// The nine mapped moments (Eq. mapping_nine_targets): [rho, rho u, rho v,
// rho E, G_xx, G_yy, G_xy, J_x, J_y] with E = (|xi|^2 g + h)/2, G the second g
// moments and J = sum w xi E.  The first four are the four-moment set.
__device__ __forceinline__ void acc_m9(double* m, double w, double x, double y, double g, double h) {
    const double wg = w * g, E = 0.5 * w * ((x * x + y * y) * g + h);
    m[0] += wg; m[1] += wg * x; m[2] += wg * y; m[3] += E;
    m[4] += wg * x * x; m[5] += wg * y * y; m[6] += wg * x * y; m[7] += E * x; m[8] += E * y;
}

// Coefficients of the linear correction on level D for the moment defect dM:
// four moments (Eqs. raw_four_g_basis, raw_four_gh_coupling): dg = a . [1, x,
// y, |xi|^2], dh = (3 - D + K) R T_tar dg; nine moments (Eqs. raw_six_g_basis,
// raw_three_h_basis, mapping_h_residual_correction): dg = a . [1, x, y, x^2,
// y^2, xy] against the six g moments, then dh = b . [1, x, y] against the
// energy and energy-flux residuals left by dg.
struct MapCoef { double a[6], b[3]; bool nine; };

// Exponential moment-constrained correction (Sec. 3.3, Eq.
// exponential_moment_correction) of a provisional pair held in the rows:
// g* = g^p e^{a.phi}, h* = h^p e^{a.phi}, phi = [1, x, y, x^2 + y^2], with a
// from Newton's method from a = 0 on the four conserved moments
// F_k(a) = sum w (psi_k g^p + psi^h_k h^p) e^{a.phi} - tgt_k, psi = [1, x, y,
// |xi|^2/2], psi^h = [0, 0, 0, 1/2], Jacobian J_km = sum w (psi_k g^p +
// psi^h_k h^p) e^{a.phi} phi_m.  Converged when every |F_k| <= 1e-14 S_k, S_k
// the sum of the terms' magnitudes; then the rows are rewritten and true is
// returned; otherwise (after EXP_MAXIT steps) the rows are left as they were.
constexpr int EXP_MAXIT = 30;
// Band of the positivity check, relative to max |g^p| of the row: values
// above -band count as nonnegative.  A tolerance of the check, not a rounding
// bound (two implementations of the step agree far closer than 1e-10 of the
// row's peak after many steps).  The same band with float rows: a float
// provisional value is rounded to about 6e-8 of itself, far below the band
// except where a large provisional value and its correction cancel to near
// zero.
constexpr double POS_EPS = 1e-10;
template <typename S>
__device__ bool map_exp(const LevelDesc& D, gptr<S> gdst, gptr<S> hdst, const double* tgt) {
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    bool ok = false;
    for (int it = 0; it <= EXP_MAXIT; ++it) {
        double s[24];                      // F[4], S[4], J[4][4]
#pragma unroll
        for (int k = 0; k < 24; ++k) s[k] = 0.0;
        for (int i = lane_id(); i < D.N; i += WL) {
            const double x = gp(D.xi_x)[i], y = gp(D.xi_y)[i], w = gp(D.w)[i];
            const double x2 = x * x + y * y;
            const double e = exp(a[0] + a[1] * x + a[2] * y + a[3] * x2);
            const double wg = w * (double)gdst[i] * e, wh = w * (double)hdst[i] * e;
            const double k4[4] = {wg, wg * x, wg * y, 0.5 * x2 * wg + 0.5 * wh};
            const double ph4[4] = {1.0, x, y, x2};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                s[k] += k4[k];
                s[4 + k] += fabs(k4[k]);
#pragma unroll
                for (int mm = 0; mm < 4; ++mm) s[8 + 4 * k + mm] += k4[k] * ph4[mm];
            }
        }
        wave_sum<24>(s);
        double F[4], J[4][4];
        bool conv = true;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            F[k] = s[k] - tgt[k];
            conv = conv && fabs(F[k]) <= 1e-14 * s[4 + k];
#pragma unroll
            for (int mm = 0; mm < 4; ++mm) J[k][mm] = s[8 + 4 * k + mm];
        }
        if (conv) { ok = true; break; }
        if (it == EXP_MAXIT) break;
        solve_fixed<4>(J, F);
#pragma unroll
        for (int k = 0; k < 4; ++k) a[k] = uni(a[k] - F[k]);
    }
    if (!ok) return false;
    for (int i = lane_id(); i < D.N; i += WL) {
        const double x = gp(D.xi_x)[i], y = gp(D.xi_y)[i];
        const double e = exp(a[0] + a[1] * x + a[2] * y + a[3] * (x * x + y * y));
        gdst[i] = (S)((double)gdst[i] * e);
        hdst[i] = (S)((double)hdst[i] * e);
    }
    return true;
}

__device__ __forceinline__ MapCoef map_coeffs(const LevelDesc& D, const double* dM, double Ttar, const Phys& ph) {
    MapCoef m{};
    m.nine = ph.map_moments == 9;
    if (m.nine) {
        const double d6[6] = {dM[0], dM[1], dM[2], dM[4], dM[5], dM[6]};
        for (int r = 0; r < 6; ++r) {
            double s = 0.0;
            for (int c = 0; c < 6; ++c) s += D.G6inv[r * 6 + c] * d6[c];
            m.a[r] = s;
        }
        double r3[3];
        for (int r = 0; r < 3; ++r) {
            double s = 0.0;
            for (int c = 0; c < 6; ++c) s += D.B36[r * 6 + c] * m.a[c];
            r3[r] = (r == 0 ? dM[3] : dM[6 + r]) - 0.5 * s;
        }
        for (int r = 0; r < 3; ++r) {
            double s = 0.0;
            for (int c = 0; c < 3; ++c) s += D.H3inv[r * 3 + c] * r3[c];
            m.b[r] = s;
        }
    } else {
        const double cK = 3.0 - ph.D + ph.K;
        const double rhs[4] = {dM[0], dM[1], dM[2], dM[3] - 0.5 * cK * ph.R * Ttar * dM[0]};
        for (int r = 0; r < 4; ++r) {
            double s = 0.0;
            for (int c = 0; c < 4; ++c) s += D.Minv[r * 4 + c] * rhs[c];
            m.a[r] = s;
        }
        m.b[0] = cK * ph.R * Ttar;         // dh = b0 dg
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) m.a[k] = uni(m.a[k]);
#pragma unroll
    for (int k = 0; k < 3; ++k) m.b[k] = uni(m.b[k]);
    return m;
}

__device__ __forceinline__ void map_delta(const MapCoef& m, double x, double y, double& dg, double& dh) {
    if (m.nine) {
        dg = m.a[0] + m.a[1] * x + m.a[2] * y + m.a[3] * x * x + m.a[4] * y * y + m.a[5] * x * y;
        dh = m.b[0] + m.b[1] * x + m.b[2] * y;
    } else {
        dg = m.a[0] + m.a[1] * x + m.a[2] * y + m.a[3] * (x * x + y * y);
        dh = m.b[0] * dg;
    }
}

template <typename S>
__device__ __forceinline__ void map_correct_apply(const LevelDesc& D, gptr<S> gdst, gptr<S> hdst, const double* dM,
                                                  const double* tgt, double Ttar, const Phys& ph, int& negflag,
                                                  unsigned long long* cnt) {
    const MapCoef mc = map_coeffs(D, dM, Ttar, ph);
    if (ph.positivity) {
        // positivity check of the linear result before it is written: a
        // nonnegative provisional g turned negative takes the exponential
        // correction (the rows still hold the provisional pair); values
        // within the band of zero count as zero
        double v[3] = {0.0, -1e300, -1e300};      // max |g^p|, -min g^p, -min g_lin
        for (int i = lane_id(); i < D.N; i += WL) {
            double dg, dh;
            map_delta(mc, gp(D.xi_x)[i], gp(D.xi_y)[i], dg, dh);
            const S gprov = gdst[i];
            v[0] = fmax(v[0], fabs((double)gprov));
            v[1] = fmax(v[1], -(double)gprov);
            v[2] = fmax(v[2], -(double)(S)((double)gprov + dg));
        }
        wave_max<3>(v);
        const double eps = POS_EPS * v[0];
        if (v[1] <= eps && v[2] > eps) {
            negflag = 1;
            const bool ok = map_exp<S>(D, gdst, hdst, tgt);
            if (lane_id() == 0) atomicAdd(cnt + (ok ? 1 : 2), 1ull);
            if (ok) return;
        }
    }
    for (int i = lane_id(); i < D.N; i += WL) {
        const double x = gp(D.xi_x)[i], y = gp(D.xi_y)[i];
        double dg, dh;
        map_delta(mc, x, y, dg, dh);
        const S gprov = gdst[i];
        const S gn = (S)((double)gprov + dg);
        if (gn < S(0) && gprov >= S(0)) negflag = 1;
        gdst[i] = gn;
        hdst[i] = (S)((double)hdst[i] + dh);
    }
}

// Items [first, n) with stride `stride` (one wave per item): the loop of the
// kernel below, and one stage of the persistent step.
template <typename S>
__device__ __forceinline__ void ghost_items(const LevelDesc* __restrict__ lvs, const GhostItem* __restrict__ items,
                                            int n, const int* __restrict__ cell_lev,
                                            const int* __restrict__ cell_slot, const double* __restrict__ params,
                                            Phys ph, unsigned long long* neg, int first, int stride) {
    for (int it = first; it < n; it += stride) {
        const GhostItem G = items[it];
        const LevelDesc& Ls = lvs[cell_lev[G.n]];
        const LevelDesc& Ld = lvs[G.dst];
        const size_t srow = (size_t)cell_slot[G.n] * Ls.stride;
        auto sg = rowp<S>(Ls.fg, srow);
        auto sh = rowp<S>(Ls.fh, srow);
        auto dg = rowp<S>(Ld.fg, (size_t)(Ld.n_rows_state + G.row) * Ld.stride);
        auto dh = rowp<S>(Ld.fh, (size_t)(Ld.n_rows_state + G.row) * Ld.stride);
        double m[18];
#pragma unroll
        for (int k = 0; k < 18; ++k) m[k] = 0.0;
        for (int i = lane_id(); i < Ls.N; i += WL)         // target: moments on the source level
            acc_m9(m, gp(Ls.w)[i], gp(Ls.xi_x)[i], gp(Ls.xi_y)[i], (double)sg[i], (double)sh[i]);
        for (int P = lane_id(); P < Ld.N; P += WL) {       // provisional projection
            double gP = 0.0, HP = 0.0;
            for (int e = gp(G.tab.off)[P]; e < gp(G.tab.off)[P + 1]; ++e) {
                const int a = gp(G.tab.idx)[e];
                const double fr = gp(G.tab.frac)[e];
                const double ga = (double)sg[a];
                const double xa = gp(Ls.xi_x)[a], ya = gp(Ls.xi_y)[a];
                gP += fr * ga;
                HP += fr * ((double)sh[a] + (xa * xa + ya * ya) * ga);
            }
            const double x = gp(Ld.xi_x)[P], y = gp(Ld.xi_y)[P], w = gp(Ld.w)[P];
            const double hP = HP - (x * x + y * y) * gP;
            const S gs = (S)gP, hs = (S)hP;
            dg[P] = gs;
            dh[P] = hs;
            acc_m9(m + 9, w, x, y, (double)gs, (double)hs);
        }
        wave_sum<18>(m);
        int nf = 0;
        if (ph.map_moments) {
            double dM[9];
            for (int k = 0; k < 9; ++k) dM[k] = m[k] - m[9 + k];
            map_correct_apply<S>(Ld, dg, dh, dM, m, params[(size_t)G.n * NPARAM + P_T], ph, nf, neg);
        }
        nf = __any(nf);
        if (lane_id() == 0 && nf) atomicAdd(neg, 1ull);
    }
}

template <typename S>
__global__ __launch_bounds__(BS) void k_ghost(const LevelDesc* __restrict__ lvs, const GhostItem* __restrict__ items,
                                              int n, const int* __restrict__ cell_lev,
                                              const int* __restrict__ cell_slot, const double* __restrict__ params,
                                              Phys ph, unsigned long long* neg) {
    ghost_items<S>(lvs, items, n, cell_lev, cell_slot, params, ph, neg, item0(), istride());
}

// ---------------------------------------------------------------------------
// same-level faces
// ---------------------------------------------------------------------------
// van Leer's limited slope from two one-sided slopes: 2ab/(a+b) where they
// agree in sign, else 0.  Written without a branch (the division runs on every
// lane with a safe denominator) so the stencil loads around it stay batched.
__device__ __forceinline__ double vl_div(double n, double d) { return n / d; }
__device__ __forceinline__ float vl_div(float n, float d) { return n * __builtin_amdgcn_rcpf(d); }
template <typename C>
__device__ __forceinline__ C van_leer(C a, C b) {
    const C p = a * b;
    const bool pos = p > C(0);
    const C q = vl_div(C(2) * p, pos ? a + b : C(1));
    return pos ? q : C(0);
}

template <typename S>
struct Side {                       // one cell's reconstruction stencil on its level
    gptr<const S> base[2];          // the level's phi_bar+ buffers (g, h)
    size_t off[5];                  // element offsets of the rows: own, W, E, S, N
    S G[4], id[4];                  // [t_i; t_j]^-1 and 1/|x_n - x_c|
    S dx, dy;                       // x_f - x_cell
};

// Row of a neighbour code: same-level cell, ghost row after the level's cells,
// or the cell's own row when there is no neighbour (zero one-sided difference).
__device__ __forceinline__ size_t nb_off(const LevelDesc& L, int code, const int* cell_slot, size_t own) {
    if (code == -1) return own;
    if (code >= 0) return (size_t)cell_slot[code] * L.stride;
    return (size_t)(L.n_rows_state + (-2 - code)) * L.stride;
}

template <typename S>
__device__ __forceinline__ void load_side(Side<S>& sd, const LevelDesc& L, int cell, const int* cell_slot,
                                          const int* cell_nbr, const CellGeom* geom, double dx, double dy) {
    sd.base[0] = gp(reinterpret_cast<const S*>(L.fg));
    sd.base[1] = gp(reinterpret_cast<const S*>(L.fh));
    const size_t own = (size_t)cell_slot[cell] * L.stride;
    sd.off[0] = own;
#pragma unroll
    for (int k = 0; k < 4; ++k) sd.off[k + 1] = nb_off(L, cell_nbr[4 * cell + k], cell_slot, own);
    const CellGeom& gm = geom[cell];
#pragma unroll
    for (int k = 0; k < 4; ++k) { sd.G[k] = (S)gm.G[k]; sd.id[k] = (S)gm.inv_dist[k]; }
    sd.dx = (S)dx; sd.dy = (S)dy;
}

// Per-lane choice between two stencils of the same level (branch-free upwind selection).
template <typename S>
__device__ __forceinline__ void select_side(Side<S>& o, const Side<S>& a, const Side<S>& b, bool useA) {
    o.base[0] = a.base[0];
    o.base[1] = a.base[1];
#pragma unroll
    for (int k = 0; k < 5; ++k) o.off[k] = useA ? a.off[k] : b.off[k];
#pragma unroll
    for (int k = 0; k < 4; ++k) { o.G[k] = useA ? a.G[k] : b.G[k]; o.id[k] = useA ? a.id[k] : b.id[k]; }
    o.dx = useA ? a.dx : b.dx;
    o.dy = useA ? a.dy : b.dy;
}

// Limited gradient of phi_bar+ at velocity index i: per index direction a van
// Leer limited pair of one-sided slopes, mapped through [t_i; t_j]^-1.
template <typename S>
__device__ __forceinline__ void side_slope(const Side<S>& sd, int i, S (&f)[2], S (&sx)[2], S (&sy)[2]) {
#pragma unroll
    for (int comp = 0; comp < 2; ++comp) {
        const auto B = sd.base[comp] + i;
        const S fv = B[sd.off[0]];
        S sl[2];
#pragma unroll
        for (int d = 0; d < 2; ++d) {
            const S a = (fv - B[sd.off[1 + 2 * d]]) * sd.id[2 * d];
            const S b = (B[sd.off[2 + 2 * d]] - fv) * sd.id[2 * d + 1];
            sl[d] = van_leer<S>(a, b);
        }
        f[comp] = fv;
        sx[comp] = sd.G[0] * sl[0] + sd.G[1] * sl[1];
        sy[comp] = sd.G[2] * sl[0] + sd.G[3] * sl[1];
    }
}

// phi_bar+ of the side's cell extrapolated to the face at velocity index i:
// phi_bar+ + (x_f - x_c - xi s) . sigma.
template <typename S>
__device__ __forceinline__ void side_ext(const Side<S>& sd, int i, S x, S y, S s, S& eg, S& eh) {
    S f[2], sx[2], sy[2];
    side_slope<S>(sd, i, f, sx, sy);
    const S ax = sd.dx - x * s, ay = sd.dy - y * s;
    eg = f[0] + ax * sx[0] + ay * sy[0];
    eh = f[1] + ax * sx[1] + ay * sy[1];
}

// Face state from the reduced raw moments of phi_bar_f (Eq. W_from_bar,
// q_f = 2 tau_f q_bar / (2 tau_f + s Pr)), the compatibility coefficients of
// the face target, and the recovery weights c1 = 2 tau_f/(2 tau_f + s),
// c2 = s/(2 tau_f + s) of Eq. recover_phi.  Returns the target in double.
template <typename S, int U>
__device__ __forceinline__ Eq<double> face_target(const LevelDesc& L, double* m, double u0, double v0,
                                                  const Phys& ph, bool compat, double& c1, double& c2,
                                                  double* Tout = nullptr) {
    double rho, u, v, T, qx, qy;
    raw_to_state(m, u0, v0, ph, rho, u, v, T, qx, qy);
    const double s = 0.5 * ph.dt;
    const double tau = viscosity(T, ph) / (rho * ph.R * T);
    qx = 2.0 * tau * qx / (2.0 * tau + s * ph.Pr);
    qy = 2.0 * tau * qy / (2.0 * tau + s * ph.Pr);
    double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (compat) {
        const Eq<S> eu = eq_cast<S>(make_eq(rho, u, v, T, qx, qy, nullptr, ph));
        compat_solve_any<S, U>(L, eu, rho, u, v, T, qx, qy, ph, a);
    }
    c1 = 2.0 * tau / (2.0 * tau + s);
    c2 = s / (2.0 * tau + s);
    if (Tout) *Tout = T;
    return make_eq(rho, u, v, T, qx, qy, compat ? a : nullptr, ph);
}

// The five stencil values (own, W, E, S, N) of g and h at one velocity index,
// from side a or b chosen per lane.
template <typename S>
struct Stencil { S v[2][5]; };

template <typename S, typename SD>
__device__ __forceinline__ void load_stencil(const SD& a, const SD& b, bool useA, int i, Stencil<S>& st) {
#pragma unroll
    for (int comp = 0; comp < 2; ++comp) {
        const auto B = a.base[comp] + i;
#pragma unroll
        for (int k = 0; k < 5; ++k) st.v[comp][k] = B[useA ? a.off[k] : b.off[k]];
    }
}

// phi_bar+ + (x_f - x_c - xi s) . sigma from a loaded stencil (Eqs.
// bar_phi_transport, reconstruction): per index direction a van Leer limited
// pair of one-sided slopes, mapped through [t_i; t_j]^-1.
template <typename S>
__device__ __forceinline__ void stencil_ext(const Side<S>& a, const Side<S>& b, bool useA, const Stencil<S>& st,
                                            S x, S y, S s, S& eg, S& eh) {
    S G[4], id[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) { G[k] = useA ? a.G[k] : b.G[k]; id[k] = useA ? a.id[k] : b.id[k]; }
    const S ax = (useA ? a.dx : b.dx) - x * s, ay = (useA ? a.dy : b.dy) - y * s;
    S e[2];
#pragma unroll
    for (int comp = 0; comp < 2; ++comp) {
        const S fv = st.v[comp][0];
        const S s0 = van_leer<S>((fv - st.v[comp][1]) * id[0], (st.v[comp][2] - fv) * id[1]);
        const S s1 = van_leer<S>((fv - st.v[comp][3]) * id[2], (st.v[comp][4] - fv) * id[3]);
        e[comp] = fv + ax * (G[0] * s0 + G[1] * s1) + ay * (G[2] * s0 + G[3] * s1);
    }
    eg = e[0];
    eh = e[1];
}

// Face state from the raw moments of phi_bar_f (Eq. W_from_bar): W_f, tau_f,
// q_f = 2 tau_f q_bar/(2 tau_f + s Pr) and the recovery weights c1 = 2 tau_f /
// (2 tau_f + s), c2 = s/(2 tau_f + s) of Eq. recover_phi (one lane per face).
struct FaceState { double rho, u, v, T, qx, qy, c1, c2; };

__device__ __forceinline__ FaceState face_state(const double* mm, double u0, double v0, const Phys& ph) {
    double m[11];
#pragma unroll
    for (int k = 0; k < 11; ++k) m[k] = mm[k];
    FaceState f;
    raw_to_state(m, u0, v0, ph, f.rho, f.u, f.v, f.T, f.qx, f.qy);
    const double s = 0.5 * ph.dt;
    const double tau = viscosity(f.T, ph) / (f.rho * ph.R * f.T);
    f.qx = 2.0 * tau * f.qx / (2.0 * tau + s * ph.Pr);
    f.qy = 2.0 * tau * f.qy / (2.0 * tau + s * ph.Pr);
    f.c1 = 2.0 * tau / (2.0 * tau + s);
    f.c2 = s / (2.0 * tau + s);
    return f;
}

// The same with one side for the whole wavefront (no per-lane choice).
template <typename S, typename SD>
__device__ __forceinline__ void load_stencil1(const SD& a, int i, Stencil<S>& st) {
#pragma unroll
    for (int comp = 0; comp < 2; ++comp) {
        const auto B = a.base[comp] + i;
#pragma unroll
        for (int k = 0; k < 5; ++k) st.v[comp][k] = B[a.off[k]];
    }
}

template <typename S>
__device__ __forceinline__ void stencil_ext1(const Side<S>& a, const Stencil<S>& st, S x, S y, S s, S& eg, S& eh) {
    const S ax = a.dx - x * s, ay = a.dy - y * s;
    S e[2];
#pragma unroll
    for (int comp = 0; comp < 2; ++comp) {
        const S fv = st.v[comp][0];
        const S s0 = van_leer<S>((fv - st.v[comp][1]) * a.id[0], (st.v[comp][2] - fv) * a.id[1]);
        const S s1 = van_leer<S>((fv - st.v[comp][3]) * a.id[2], (st.v[comp][4] - fv) * a.id[3]);
        e[comp] = fv + ax * (a.G[0] * s0 + a.G[1] * s1) + ay * (a.G[2] * s0 + a.G[3] * s1);
    }
    eg = e[0];
    eh = e[1];
}

// ---------------------------------------------------------------------------
// Unstructured meshes (triangles and quadrilaterals): the stencil is the cell
// and its face neighbours (slot k = the cell's k-th edge; a missing neighbour
// reads the cell's own row, a zero difference).  The gradient is the least-
// squares fit over the face neighbours, a boundary face adding a zero-gradient
// ghost at the mirror point (its weight sits in the precomputed coefficients),
// limited by psi = min(1, min over faces of V(d+, d-)) with Venkatakrishnan's
// V(d+, d-) = (d+^2 + eps^2 + 2 d- d+) / (d+^2 + 2 d-^2 + d- d+ + eps^2),
// d- = grad . (x_f - x_c), d+ the largest (d- > 0) or smallest (d- < 0)
// neighbour difference including zero; faces with d- = 0 impose nothing.
// eps^2 = |V_c|^(3/2) phi_ref^2, phi_ref the largest |phi| of the stencil
// (relative, since distribution values span many orders of magnitude).
// ---------------------------------------------------------------------------
template <typename S>
struct USide {
    gptr<const S> base[2];
    size_t off[5];                  // own row, then the four slots
    S lx[4], ly[4];                 // least-squares coefficients per slot
    S fx[4], fy[4];                 // x_f - x_c per slot (0: no face)
    S eps2;                         // |V_c|^(3/2), to be scaled by phi_ref^2
    S dx, dy;                       // x_f - x_cell of the face being reconstructed
};

template <typename S>
__device__ __forceinline__ void load_side(USide<S>& sd, const LevelDesc& L, int cell, const int* cell_slot,
                                          const int* cell_nbr, const CellGeom* geom, double dx, double dy) {
    sd.base[0] = gp(reinterpret_cast<const S*>(L.fg));
    sd.base[1] = gp(reinterpret_cast<const S*>(L.fh));
    const size_t own = (size_t)cell_slot[cell] * L.stride;
    sd.off[0] = own;
#pragma unroll
    for (int k = 0; k < 4; ++k) sd.off[k + 1] = nb_off(L, cell_nbr[4 * cell + k], cell_slot, own);
    const CellGeom& gm = geom[cell];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        sd.lx[k] = (S)gm.lx[k]; sd.ly[k] = (S)gm.ly[k];
        sd.fx[k] = (S)gm.fox[k]; sd.fy[k] = (S)gm.foy[k];
    }
    sd.eps2 = (S)gm.eps2;
    sd.dx = (S)dx; sd.dy = (S)dy;
}

// Limited gradient (sx, sy) from the stencil values v (own, slots 0..3).  The
// smallest V is tracked as a fraction (cross-multiplied compares, positive
// denominators), so one division gives psi.
template <typename S>
__device__ __forceinline__ void venkat_slope(const S (&lx)[4], const S (&ly)[4], const S (&fx)[4], const S (&fy)[4],
                                             S eps2, const S (&v)[5], S& sx, S& sy) {
    const S fc = v[0];
    S gx = S(0), gy = S(0), dmax = S(0), dmin = S(0), ref = fabs(fc);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const S d = v[k + 1] - fc;
        gx += lx[k] * d;
        gy += ly[k] * d;
        dmax = d > dmax ? d : dmax;
        dmin = d < dmin ? d : dmin;
        ref = fmax(ref, fabs(v[k + 1]));
    }
    eps2 = eps2 * ref * ref;
    S bn = S(1), bd = S(1);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const S dm = gx * fx[k] + gy * fy[k];
        const S dp = dm > S(0) ? dmax : dmin;
        const S num = dp * dp + eps2 + S(2) * dm * dp;
        const S den = dp * dp + S(2) * dm * dm + dm * dp + eps2;
        if (dm != S(0) && num * bd < bn * den) { bn = num; bd = den; }
    }
    const S psi = bn / bd;
    sx = psi * gx;
    sy = psi * gy;
}

template <typename S>
__device__ __forceinline__ void side_slope(const USide<S>& sd, int i, S (&f)[2], S (&sx)[2], S (&sy)[2]) {
#pragma unroll
    for (int comp = 0; comp < 2; ++comp) {
        const auto B = sd.base[comp] + i;
        S v[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) v[k] = B[sd.off[k]];
        f[comp] = v[0];
        venkat_slope<S>(sd.lx, sd.ly, sd.fx, sd.fy, sd.eps2, v, sx[comp], sy[comp]);
    }
}

template <typename S>
__device__ __forceinline__ void stencil_ext(const USide<S>& a, const USide<S>& b, bool useA, const Stencil<S>& st,
                                            S x, S y, S s, S& eg, S& eh) {
    S lx[4], ly[4], fx[4], fy[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        lx[k] = useA ? a.lx[k] : b.lx[k]; ly[k] = useA ? a.ly[k] : b.ly[k];
        fx[k] = useA ? a.fx[k] : b.fx[k]; fy[k] = useA ? a.fy[k] : b.fy[k];
    }
    const S eps2 = useA ? a.eps2 : b.eps2;
    const S ax = (useA ? a.dx : b.dx) - x * s, ay = (useA ? a.dy : b.dy) - y * s;
    S e[2];
#pragma unroll
    for (int comp = 0; comp < 2; ++comp) {
        S sx, sy;
        venkat_slope<S>(lx, ly, fx, fy, eps2, st.v[comp], sx, sy);
        e[comp] = st.v[comp][0] + ax * sx + ay * sy;
    }
    eg = e[0];
    eh = e[1];
}

template <typename S>
__device__ __forceinline__ void stencil_ext1(const USide<S>& a, const Stencil<S>& st, S x, S y, S s, S& eg, S& eh) {
    const S ax = a.dx - x * s, ay = a.dy - y * s;
    S e[2];
#pragma unroll
    for (int comp = 0; comp < 2; ++comp) {
        S sx, sy;
        venkat_slope<S>(a.lx, a.ly, a.fx, a.fy, a.eps2, st.v[comp], sx, sy);
        e[comp] = st.v[comp][0] + ax * sx + ay * sy;
    }
    eg = e[0];
    eh = e[1];
}

// The side type of a mesh kind (0 structured, 1 unstructured).
template <typename S, int MK>
using SideOf = typename std::conditional<MK == 1, USide<S>, Side<S>>::type;

// Face stage, part 1 (reconstruction): for every same-level interior face and
// every boundary face, the interface value phi_bar_f = phi_bar+_up + (x_f -
// x_up - xi s) . sigma_up (both sides averaged where xi . n = 0) is written to
// the face row.  Interior faces also reduce the eleven raw moments of phi_bar_f
// (about the mean of the two cell velocities); boundary faces reduce the
// outgoing mass flux.  Per-face results go to fmom[item][NFMOM] (the moments,
// then the velocity shift they are taken about).
template <typename S, int U, int MK>
__device__ __forceinline__ void face_rec_points(const LevelDesc& L, const FaceItem& F, const int* cell_slot,
                                                const int* cell_nbr, const CellGeom* geom, const double* params,
                                                const Phys& ph, int beg, int N, double (&m)[11], double& u0,
                                                double& v0) {
    const S s = (S)(0.5 * ph.dt);
    auto rg = rowp<S>(L.Fg, (size_t)F.row * L.stride);
    auto rh = rowp<S>(L.Fh, (size_t)F.row * L.stride);
    SideOf<S, MK> sL;
    load_side<S>(sL, L, F.L, cell_slot, cell_nbr, geom, F.dLx, F.dLy);
    const bool interior = F.R >= 0;
    SideOf<S, MK> sR = sL;
    u0 = 0.0;
    v0 = 0.0;
    if (interior) {
        load_side<S>(sR, L, F.R, cell_slot, cell_nbr, geom, F.dRx, F.dRy);
        u0 = 0.5 * (params[(size_t)F.L * NPARAM + P_U] + params[(size_t)F.R * NPARAM + P_U]);
        v0 = 0.5 * (params[(size_t)F.L * NPARAM + P_V] + params[(size_t)F.R * NPARAM + P_V]);
    }
#pragma unroll
    for (int k = 0; k < 11; ++k) m[k] = 0.0;
    for (int i0 = beg + lane_id(); i0 < N; i0 += WL * U) {
        double xv[U], yv[U], wv[U];
        bool up[U];
        // points are stored by velocity angle, so a chunk almost always has
        // one upwind side for the whole wavefront: then that side's stencil
        // is used with scalar offsets and coefficients
        bool allL = true, allR = true;
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int i = i0 + q * WL, ic = clampi(i, N);
            load_xy<S>(L, ic, xv[q], yv[q]);
            wv[q] = i < N ? gp(L.w)[ic] : 0.0;
            const double dn = xv[q] * F.nx + yv[q] * F.ny;
            up[q] = dn >= 0.0;
            allL = allL && (i >= N || dn > 0.0);
            allR = allR && (i >= N || dn < 0.0);
        }
        const int side = !interior ? 0 : (__all(allL) ? 0 : (__all(allR) ? 1 : 2));
        S eg[U], eh[U];
        if (side < 2) {
            const SideOf<S, MK>& sd = side == 0 ? sL : sR;
            Stencil<S> st[U];
#pragma unroll
            for (int q = 0; q < U; ++q) load_stencil1<S>(sd, clampi(i0 + q * WL, N), st[q]);
#pragma unroll
            for (int q = 0; q < U; ++q) stencil_ext1<S>(sd, st[q], (S)xv[q], (S)yv[q], s, eg[q], eh[q]);
        } else {
            Stencil<S> st[U];
#pragma unroll
            for (int q = 0; q < U; ++q) load_stencil<S>(sL, sR, up[q], clampi(i0 + q * WL, N), st[q]);
#pragma unroll
            for (int q = 0; q < U; ++q) {
                const int ic = clampi(i0 + q * WL, N);
                const S x = (S)xv[q], y = (S)yv[q];
                stencil_ext<S>(sL, sR, up[q], st[q], x, y, s, eg[q], eh[q]);
                const double dn = xv[q] * F.nx + yv[q] * F.ny;
                if (dn == 0.0) {                    // both sides, averaged
                    Stencil<S> sb;
                    load_stencil<S>(sL, sR, false, ic, sb);
                    S bg, bh;
                    stencil_ext<S>(sL, sR, false, sb, x, y, s, bg, bh);
                    eg[q] = S(0.5) * (eg[q] + bg);
                    eh[q] = S(0.5) * (eh[q] + bh);
                }
            }
        }
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int i = i0 + q * WL;
            if (i < N) { rg[i] = eg[q]; rh[i] = eh[q]; }
            if (interior) {
                acc_raw<S>(m, wv[q], xv[q] - u0, yv[q] - v0, eg[q], eh[q]);
            } else {
                // the outgoing mass flux in the update's own arithmetic (double
                // velocities), so that a diffuse wall's zero net mass flux holds
                // in the update for either storage precision
                const int ic = clampi(i0 + q * WL, N);
                const double dn = gp(L.xi_x)[ic] * F.nx + gp(L.xi_y)[ic] * F.ny;
                if (dn > 0) m[0] += wv[q] * dn * (double)eg[q];
            }
        }
    }
}

template <typename S, int U, int MINW, int MK>
__global__ __launch_bounds__(BS, MINW) void k_face_rec(const LevelDesc* __restrict__ lvs,
                                                       const FaceItem* __restrict__ items, int nF,
                                                       const int* __restrict__ cell_slot,
                                                       const int* __restrict__ cell_nbr,
                                                       const CellGeom* __restrict__ geom,
                                                       const double* __restrict__ params, Phys ph,
                                                       double* __restrict__ fmom, int CH, int nch) {
    const int n = nF * nch;
    for (int it = item0(); it < n; it += istride()) {
        const int kc = it / nF, f = it - kc * nF;
        const FaceItem F = items[f];
        const LevelDesc& L = lvs[F.lev];
        const int beg = kc * CH;
        if (beg >= L.N) continue;
        const int N = min(L.N, beg + CH);      // end of this chunk
        double m[11], u0, v0;
        face_rec_points<S, U, MK>(L, F, cell_slot, cell_nbr, geom, params, ph, beg, N, m, u0, v0);
        double* out = fmom + (size_t)it * NFMOM;
        wave_sum<11>(m);
        if (lane_id() < 11) {
#pragma unroll
            for (int k = 0; k < 11; ++k)
                if (lane_id() == k) out[k] = m[k];
        }
        if (lane_id() == 0) { out[11] = u0; out[12] = v0; }
    }
}

// Face stage, part 2 (target), staged as the cell stage, for the same faces:
//  (lane per face) the face state and the uncorrected target;
//  (wave per face) the compatibility sums of the target; for a diffuse wall
//     the incoming mass flux of the wall Maxwellian;
//  (lane per face) the record the update needs to finish F = A_f (xi . n)
//     phi_f at every velocity (layout FP_*).  Interior faces: corrected target
//     and recovery weights (Eq. recover_phi).  Boundary faces (outward normal):
//     outgoing velocities carry the reconstruction, incoming ones the boundary
//     state -- diffuse wall rho_w g_eq(u_w, T_w) with rho_w from zero net mass
//     flux, far-field Maxwellian, or the cell's phi_bar+ (zero-gradient
//     outflow).
// Incoming mass flux sum w (xi . n) g_w over xi . n < 0 of a diffuse wall's
// Maxwellian es (unit density), in one wave (every lane holds the result).
template <typename S, int U>
__device__ __forceinline__ double wall_inflow(const LevelDesc& L, const FaceItem& F, const Eq<S>& es) {
    const int N = L.N;
    double m1[1] = {0.0};
    for (int i0 = lane_id(); i0 < N; i0 += WL * U) {
        double xv[U], yv[U], wv[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int i = i0 + q * WL, ic = clampi(i, N);
            xv[q] = gp(L.xi_x)[ic]; yv[q] = gp(L.xi_y)[ic];
            wv[q] = i < N ? gp(L.w)[ic] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const double dn = xv[q] * F.nx + yv[q] * F.ny;
            if (dn < 0) {
                S gs, hs;
                eq_eval<S>(es, (S)xv[q], (S)yv[q], gs, hs);
                m1[0] += wv[q] * dn * (double)gs;
            }
        }
    }
    wave_sum<1>(m1);
    return m1[0];
}

// The record the update reads for one face (layout FP_*).
__device__ __forceinline__ void write_face_record(double* o, double kind, const FaceItem& F, double c1, double c2,
                                                  const Eq<double>& e) {
    o[FP_KIND] = kind; o[FP_ROW] = (double)F.row; o[FP_NX] = F.nx; o[FP_NY] = F.ny;
    o[FP_C1] = c1; o[FP_C2] = c2;
    o[FP_RN] = e.rn; o[FP_UX] = e.ux; o[FP_UY] = e.uy; o[FP_I2RT] = e.i2RT; o[FP_RT] = e.RT;
    o[FP_IRT] = e.iRT; o[FP_XQX] = e.Xqx; o[FP_XQY] = e.Xqy;
    o[FP_B0] = e.b0; o[FP_B1] = e.b1; o[FP_B2] = e.b2; o[FP_B3] = e.b3;
    o[FP_CORR] = e.corr ? 1.0 : 0.0;
    o[FP_E4] = e.e4; o[FP_E5] = e.e5; o[FP_E6] = e.e6; o[FP_E7] = e.e7; o[FP_CKRT] = e.cKRT;
    o[FP_C8] = e.c8 ? 1.0 : 0.0;
}

template <typename S, int U, int MINW, int CM>
__global__ __launch_bounds__(GBS, MINW) void k_face_target(const LevelDesc* __restrict__ lvs,
                                                           const FaceItem* __restrict__ items, int n,
                                                           const BCDev* __restrict__ bcs, Phys ph,
                                                           const double* __restrict__ fmom,
                                                           double* __restrict__ fpar, int CH) {
    constexpr int NS = CM == 8 ? 64 : 13;      // compatibility sums per face
    __shared__ double sh_m[GW][NS];
    __shared__ FaceState sh_f[GW];
    __shared__ Eq<double> sh_e[GW];
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));   // wave index (uniform)
    const int t = threadIdx.x;
    for (int g0 = wg_index() * GW; g0 < n; g0 += gridDim.x * GW) {
        // face state and uncorrected target
        if (t < GW && g0 + t < n) {
            const FaceItem F = items[g0 + t];
            double mm[NFMOM];
            sum_chunks(fmom, g0 + t, n, lvs[F.lev].N, CH, mm);
            sh_m[t][0] = mm[0];                       // boundary: the outgoing mass flux
            if (F.R >= 0) {
                const FaceState fs = face_state(mm, mm[11], mm[12], ph);
                sh_f[t] = fs;
                sh_e[t] = make_eq(fs.rho, fs.u, fs.v, fs.T, fs.qx, fs.qy, nullptr, ph);
            } else {
                const BCDev bc = bcs[-1 - F.R];
                FaceState fs{};
                fs.c1 = F.area;
                fs.c2 = F.area;
                sh_f[t] = fs;
                sh_e[t] = bc.kind == 2 ? make_eq(bc.rho, bc.u, bc.v, bc.T, 0.0, 0.0, nullptr, ph)
                                       : make_eq(1.0, bc.u, bc.v, bc.T, 0.0, 0.0, nullptr, ph);
            }
        }
        __syncthreads();
        // compatibility sums (interior) or the wall's incoming mass flux
        for (int kk = 0; kk < IPW; ++kk) {
            const int j = w + GWV * kk;
            const int it = g0 + j;
            if (it >= n) break;
            const FaceItem F = items[it];
            const LevelDesc& L = lvs[F.lev];
            if (F.R >= 0) {
                if (ph.compat && ph.face_compat) {
                    double sm[NS];
                    if constexpr (CM == 8) {
                        const FaceState& fs = sh_f[j];
                        compat_sums8<S, U>(L, eq_cast<S>(sh_e[j]), fs.u, fs.v, fs.T, ph, sm);
                    } else {
                        compat_sums<S, U>(L, eq_cast<S>(sh_e[j]), sm);
                    }
                    if (lane_id() < NS) {
#pragma unroll
                        for (int k = 0; k < NS; ++k)
                            if (lane_id() == k) sh_m[j][k] = sm[k];
                    }
                }
            } else if (bcs[-1 - F.R].kind == 1) {
                const double m1 = wall_inflow<S, U>(L, F, eq_cast<S>(sh_e[j]));
                if (lane_id() == 0) sh_m[j][1] = m1;      // [0] keeps the outgoing flux
            }
        }
        __syncthreads();
        // face record
        if (t < GW && g0 + t < n) {
            const FaceItem F = items[g0 + t];
            FaceState fs = sh_f[t];
            Eq<double> e = sh_e[t];
            double kind = 0.0, c1 = fs.c1, c2 = fs.c2;
            if (F.R >= 0) {
                if (ph.compat && ph.face_compat) {
                    double a[8];
                    if constexpr (CM == 8)
                        compat_from_sums8(sh_m[t], fs.rho, fs.u, fs.v, fs.T, (1.0 - ph.Pr) * fs.qx,
                                          (1.0 - ph.Pr) * fs.qy, ph, a);
                    else
                        compat_from_sums(sh_m[t], fs.rho, fs.u, fs.v, fs.T, ph, a);
                    e = make_eq(fs.rho, fs.u, fs.v, fs.T, fs.qx, fs.qy, a, ph);
                }
                c1 *= F.area;
                c2 *= F.area;
            } else {
                const BCDev bc = bcs[-1 - F.R];
                kind = (double)bc.kind;
                if (bc.kind == 1) c2 = F.area * (-sh_m[t][0] / sh_m[t][1]);
            }
            write_face_record(fpar + (size_t)(g0 + t) * NFP, kind, F, c1, c2, e);
        }
        __syncthreads();
    }
}

// Reconstruction and target of one face in one wave: all of the face's points
// in one pass, then the face state, the corrected target and the record from
// the wave's own sums (every lane holds them; lane 0 writes).  The form for
// level sets whose levels fit one velocity chunk, where the reconstruction has
// no chunk partials to add and the staged target's per-workgroup hand-overs
// would dominate.  Same arithmetic as k_face_rec + k_face_target.
template <typename S, int U, int CM, int MK>
__device__ __forceinline__ void face_full_items(const LevelDesc* __restrict__ lvs, const FaceItem* __restrict__ items,
                                                int nF, const int* __restrict__ cell_slot,
                                                const int* __restrict__ cell_nbr, const CellGeom* __restrict__ geom,
                                                const double* __restrict__ params, const BCDev* __restrict__ bcs,
                                                Phys ph, double* __restrict__ fpar, int first, int stride) {
    for (int f = first; f < nF; f += stride) {
        const FaceItem F = items[f];
        const LevelDesc& L = lvs[F.lev];
        double m[11], u0, v0;
        face_rec_points<S, U, MK>(L, F, cell_slot, cell_nbr, geom, params, ph, 0, L.N, m, u0, v0);
        wave_sum<11>(m);
        double kind = 0.0, c1, c2;
        Eq<double> e;
        if (F.R >= 0) {
            const FaceState fs = face_state(m, u0, v0, ph);
            e = make_eq(fs.rho, fs.u, fs.v, fs.T, fs.qx, fs.qy, nullptr, ph);
            if (ph.compat && ph.face_compat) {
                double a[8];
                if constexpr (CM == 8) {
                    double A[64];
                    compat_sums8<S, U>(L, eq_cast<S>(e), fs.u, fs.v, fs.T, ph, A);
                    compat_from_sums8(A, fs.rho, fs.u, fs.v, fs.T, (1.0 - ph.Pr) * fs.qx, (1.0 - ph.Pr) * fs.qy,
                                      ph, a);
                } else {
                    double sm[13];
                    compat_sums<S, U>(L, eq_cast<S>(e), sm);
                    compat_from_sums(sm, fs.rho, fs.u, fs.v, fs.T, ph, a);
                }
                e = make_eq(fs.rho, fs.u, fs.v, fs.T, fs.qx, fs.qy, a, ph);
            }
            c1 = fs.c1 * F.area;
            c2 = fs.c2 * F.area;
        } else {
            const BCDev bc = bcs[-1 - F.R];
            kind = (double)bc.kind;
            e = bc.kind == 2 ? make_eq(bc.rho, bc.u, bc.v, bc.T, 0.0, 0.0, nullptr, ph)
                             : make_eq(1.0, bc.u, bc.v, bc.T, 0.0, 0.0, nullptr, ph);
            c1 = F.area;
            c2 = F.area;
            if (bc.kind == 1) c2 = F.area * (-m[0] / wall_inflow<S, U>(L, F, eq_cast<S>(e)));
        }
        if (lane_id() == 0) write_face_record(fpar + (size_t)f * NFP, kind, F, c1, c2, e);
    }
}

template <typename S, int U, int MINW, int CM, int MK>
__global__ __launch_bounds__(BS, MINW) void k_face_full(const LevelDesc* __restrict__ lvs,
                                                        const FaceItem* __restrict__ items, int nF,
                                                        const int* __restrict__ cell_slot,
                                                        const int* __restrict__ cell_nbr,
                                                        const CellGeom* __restrict__ geom,
                                                        const double* __restrict__ params,
                                                        const BCDev* __restrict__ bcs, Phys ph,
                                                        double* __restrict__ fpar) {
    face_full_items<S, U, CM, MK>(lvs, items, nF, cell_slot, cell_nbr, geom, params, bcs, ph, fpar, item0(),
                                  istride());
}

template <typename S>
__device__ __forceinline__ Eq<S> load_face_eq(const double* fp, const Phys& ph) {
    Eq<double> d;
    d.rn = fp[FP_RN]; d.ux = fp[FP_UX]; d.uy = fp[FP_UY]; d.i2RT = fp[FP_I2RT]; d.RT = fp[FP_RT];
    d.iRT = fp[FP_IRT]; d.Xqx = fp[FP_XQX]; d.Xqy = fp[FP_XQY];
    d.b0 = fp[FP_B0]; d.b1 = fp[FP_B1]; d.b2 = fp[FP_B2]; d.b3 = fp[FP_B3];
    d.cK = ph.K + 3.0 - ph.D; d.Dp2 = ph.D + 2.0; d.Dd = ph.D; d.K2 = 2.0 * ph.K;
    d.corr = fp[FP_CORR] != 0.0;
    d.e4 = fp[FP_E4]; d.e5 = fp[FP_E5]; d.e6 = fp[FP_E6]; d.e7 = fp[FP_E7]; d.cKRT = fp[FP_CKRT];
    d.c8 = fp[FP_C8] != 0.0;
    return eq_cast<S>(d);
}

// ---------------------------------------------------------------------------
// cell update: phi~^{n+1} = 4/3 phi_bar+ - 1/3 phi~ - dt/|V| sum(+-F)
// (Eq. explicit_update).  Same-level and boundary faces are finished here from
// the face row phi_bar_f and the face record; cross-level faces arrive as final
// flux rows.  Both cells of a face evaluate the same expression on the same
// data, so the two contributions cancel exactly in the totals.  The raw moments
// of the new state (about this step's cell velocity) go to cmom for the next
// cell stage.
// Face codes (cell_frow): -1 none; else 4 x + 2 final + neg, x the face item
// (final = 0) or the level row of a final flux (final = 1).
// ---------------------------------------------------------------------------
// One cell over points [beg, N) of its level; m: the raw moments of the new
// state about the step's cell velocity (u0, v0).
template <typename S, int U>
__device__ __forceinline__ void update_points(const LevelDesc& L, int c, const int* cell_slot, const CellGeom* geom,
                                              const int* cell_frow, const FaceItem* items, const double* fpar,
                                              const double* params, const Phys& ph, int beg, int N,
                                              double (&m)[11], double& u0, double& v0) {
    const S c43 = (S)(4.0 / 3.0), c13 = (S)(1.0 / 3.0);
    const size_t row = (size_t)cell_slot[c] * L.stride;
    auto g = rowp<S>(L.g, row);
    auto h = rowp<S>(L.h, row);
    auto fg = rowp<S>(L.fg, row);
    auto fh = rowp<S>(L.fh, row);
    int code[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) code[k] = cell_frow[4 * c + k];
    const S kv = uni((S)(ph.dt / geom[c].vol));
    u0 = params[(size_t)c * NPARAM + P_U];
    v0 = params[(size_t)c * NPARAM + P_V];
#pragma unroll
    for (int k = 0; k < 11; ++k) m[k] = 0.0;
    for (int i0 = beg + lane_id(); i0 < N; i0 += WL * U) {
        double xv[U], yv[U], wv[U];
        S bg[U], bh[U], go[U], ho[U], ag[U], ah[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int i = i0 + q * WL, ic = clampi(i, N);
            xv[q] = gp(L.xi_x)[ic]; yv[q] = gp(L.xi_y)[ic];
            wv[q] = i < N ? gp(L.w)[ic] : 0.0;
            bg[q] = fg[ic]; bh[q] = fh[ic];
            go[q] = g[ic]; ho[q] = h[ic];
            ag[q] = S(0); ah[q] = S(0);
        }
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            const int cd = code[f];
            if (cd < 0) continue;
            const S sgn = (cd & 1) ? S(-1) : S(1);
            if (cd & 2) {
                const size_t r = (size_t)(cd >> 2) * L.stride;
                auto Fg = rowp<S>(L.Fg, r);
                auto Fh = rowp<S>(L.Fh, r);
                S vg[U], vh[U];
#pragma unroll
                for (int q = 0; q < U; ++q) {
                    const int ic = clampi(i0 + q * WL, N);
                    vg[q] = Fg[ic]; vh[q] = Fh[ic];
                }
#pragma unroll
                for (int q = 0; q < U; ++q) { ag[q] += sgn * vg[q]; ah[q] += sgn * vh[q]; }
                continue;
            }
            const double* fp = fpar + (size_t)(cd >> 2) * NFP;
            const int kind = __builtin_amdgcn_readfirstlane((int)fp[FP_KIND]);
            const size_t r = (size_t)items[cd >> 2].row * L.stride;
            auto Fg = rowp<S>(L.Fg, r);
            auto Fh = rowp<S>(L.Fh, r);
            const double nx = fp[FP_NX], ny = fp[FP_NY];
            const S k1 = uni((S)fp[FP_C1]), k2 = uni((S)fp[FP_C2]);
            S vg[U], vh[U];
#pragma unroll
            for (int q = 0; q < U; ++q) {
                const int ic = clampi(i0 + q * WL, N);
                vg[q] = Fg[ic]; vh[q] = Fh[ic];
            }
            if (kind == 3) {            // outflow: incoming = the cell's phi_bar+
#pragma unroll
                for (int q = 0; q < U; ++q) {
                    const double dnd = xv[q] * nx + yv[q] * ny;
                    const S dn = (S)dnd;
                    const S pg = dnd > 0 ? vg[q] : bg[q], ph_ = dnd > 0 ? vh[q] : bh[q];
                    ag[q] += sgn * (k1 * dn * pg);
                    ah[q] += sgn * (k1 * dn * ph_);
                }
                continue;
            }
            const Eq<S> e = load_face_eq<S>(fp, ph);
#pragma unroll
            for (int q = 0; q < U; ++q) {
                const double dnd = xv[q] * nx + yv[q] * ny;
                const S dn = (S)dnd;
                S gs, hs;
                eq_eval<S>(e, (S)xv[q], (S)yv[q], gs, hs);
                S pg, ph_;
                if (kind == 0) {
                    pg = k1 * vg[q] + k2 * gs;
                    ph_ = k1 * vh[q] + k2 * hs;
                } else {
                    pg = dnd > 0 ? k1 * vg[q] : k2 * gs;
                    ph_ = dnd > 0 ? k1 * vh[q] : k2 * hs;
                }
                ag[q] += sgn * (dn * pg);
                ah[q] += sgn * (dn * ph_);
            }
        }
        S gn[U], hn[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            gn[q] = c43 * bg[q] - c13 * go[q] - kv * ag[q];
            hn[q] = c43 * bh[q] - c13 * ho[q] - kv * ah[q];
        }
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int i = i0 + q * WL;
            if (i < N) { g[i] = gn[q]; h[i] = hn[q]; }
            acc_raw<S>(m, wv[q], xv[q] - u0, yv[q] - v0, gn[q], hn[q]);
        }
    }
}

template <typename S, int U, int MINW>
__global__ __launch_bounds__(BS, MINW) void k_update(const LevelDesc* __restrict__ lvs,
                                                     const int* __restrict__ cell_lev,
                                                     const int* __restrict__ cell_slot,
                                                     const int* __restrict__ order, int n_cells,
                                                     const CellGeom* __restrict__ geom,
                                                     const int* __restrict__ cell_frow,
                                                     const FaceItem* __restrict__ items,
                                                     const double* __restrict__ fpar,
                                                     const double* __restrict__ params, Phys ph,
                                                     double* __restrict__ cmom, int CH, int nch) {
    const int n = n_cells * nch;
    for (int it = item0(); it < n; it += istride()) {
        const int kc = it / n_cells, c = order[it - kc * n_cells];
        const LevelDesc& L = lvs[cell_lev[c]];
        const int beg = kc * CH;
        if (beg >= L.N) continue;
        const int N = min(L.N, beg + CH);      // end of this chunk
        double m[11], u0, v0;
        update_points<S, U>(L, c, cell_slot, geom, cell_frow, items, fpar, params, ph, beg, N, m, u0, v0);
        wave_sum<11>(m);
        if (lane_id() == 0) {
            double* o = cmom + ((size_t)kc * n_cells + c) * NMOM;
            for (int k = 0; k < 11; ++k) o[k] = m[k];
            o[M_U0] = u0;
            o[M_V0] = v0;
        }
    }
}

// The update followed, in the same wave, by the next step's cell stage for
// the same cell: the new state's moments (the wave's own sums), W, tau, q and
// the corrected target, the parameters, and the phi_bar+ row from the new
// state, which the wave re-reads point by point from what its own lanes just
// wrote.  Only the cell's own rows and parameters are touched, and no other
// cell's update reads them, so the next step's cell stage is complete when
// this launch ends.  The form for level sets whose levels fit one velocity
// chunk.  Same arithmetic as k_update + k_cell_prep.
template <typename S, int U, int CM>
__device__ __forceinline__ void update_cell_items(const LevelDesc* __restrict__ lvs, const int* __restrict__ cell_lev,
                                                  const int* __restrict__ cell_slot, const int* __restrict__ order,
                                                  int n_cells, const CellGeom* __restrict__ geom,
                                                  const int* __restrict__ cell_frow, const FaceItem* __restrict__ items,
                                                  const double* __restrict__ fpar, double* __restrict__ params,
                                                  Phys ph, double* __restrict__ cmom, int first, int stride) {
    for (int it = first; it < n_cells; it += stride) {
        const int c = order[it];
        const LevelDesc& L = lvs[cell_lev[c]];
        double cm[NMOM], u0, v0;
        double m[11];
        update_points<S, U>(L, c, cell_slot, geom, cell_frow, items, fpar, params, ph, 0, L.N, m, u0, v0);
        wave_sum<11>(m);
#pragma unroll
        for (int k = 0; k < 11; ++k) cm[k] = m[k];
        cm[M_U0] = u0;
        cm[M_V0] = v0;
        if (lane_id() == 0) {
            double* o = cmom + (size_t)c * NMOM;
            for (int k = 0; k < 11; ++k) o[k] = m[k];
            o[M_U0] = u0;
            o[M_V0] = v0;
        }
        const CellState cs = cell_state(cm, ph);
        Eq<double> e = make_eq(cs.rho, cs.u, cs.v, cs.T, cs.qx, cs.qy, nullptr, ph);
        double a[8];
        cell_target_wave<S, U, CM>(L, cs, ph, e, a);
        if (lane_id() == 0) write_params(params + (size_t)c * NPARAM, cs, a);
        phibar_points<S, U>(L, (size_t)cell_slot[c] * L.stride, e, cs.alpha, cs.beta);
    }
}

template <typename S, int U, int MINW, int CM>
__global__ __launch_bounds__(BS, MINW) void k_update_cell(const LevelDesc* __restrict__ lvs,
                                                          const int* __restrict__ cell_lev,
                                                          const int* __restrict__ cell_slot,
                                                          const int* __restrict__ order, int n_cells,
                                                          const CellGeom* __restrict__ geom,
                                                          const int* __restrict__ cell_frow,
                                                          const FaceItem* __restrict__ items,
                                                          const double* __restrict__ fpar,
                                                          double* __restrict__ params, Phys ph,
                                                          double* __restrict__ cmom) {
    update_cell_items<S, U, CM>(lvs, cell_lev, cell_slot, order, n_cells, geom, cell_frow, items, fpar, params, ph,
                                cmom, item0(), istride());
}

// ---------------------------------------------------------------------------
// diagnostics: per-cell fields and volume-weighted conserved totals
// ---------------------------------------------------------------------------
template <typename S>
__global__ __launch_bounds__(BS) void k_cell_moments(const LevelDesc* __restrict__ lvs, const int* __restrict__ cell_lev,
                                                     const int* __restrict__ cell_slot, int n_cells,
                                                     const CellGeom* __restrict__ geom, Phys ph,
                                                     double* __restrict__ out6, double* __restrict__ tot4,
                                                     double* __restrict__ out8, double* __restrict__ out3) {
    for (int c = item0(); c < n_cells; c += istride()) {
        const LevelDesc& L = lvs[cell_lev[c]];
        const size_t row = (size_t)cell_slot[c] * L.stride;
        auto g = rowp<S>(L.g, row);
        auto h = rowp<S>(L.h, row);
        double m[11];
#pragma unroll
        for (int k = 0; k < 11; ++k) m[k] = 0.0;
        for (int i = lane_id(); i < L.N; i += WL) acc_raw<S>(m, gp(L.w)[i], gp(L.xi_x)[i], gp(L.xi_y)[i], g[i], h[i]);
        wave_sum<11>(m);
        if (lane_id() == 0) {
            double rho, u, v, T, qx, qy;
            raw_to_state(m, 0.0, 0.0, ph, rho, u, v, T, qx, qy);
            const double tau = viscosity(T, ph) / (rho * ph.R * T);
            const double f = 2.0 * tau / (2.0 * tau + ph.dt * ph.Pr);
            if (out6) {
                double* o = out6 + 6 * (size_t)c;
                o[0] = rho; o[1] = u; o[2] = v; o[3] = T; o[4] = f * qx; o[5] = f * qy;
            }
            if (out8) {
                // (rho, u, v, T, qx, qy, sigma_xx, sigma_xy): deviatoric stress from
                // P_ab = sum w c_a c_b g, sigma_xx = P_xx - p
                double* o = out8 + 8 * (size_t)c;
                o[0] = rho; o[1] = u; o[2] = v; o[3] = T; o[4] = f * qx; o[5] = f * qy;
                o[6] = (m[3] - rho * u * u) - rho * ph.R * T;
                o[7] = m[4] - rho * u * v;
            }
            if (out3) {
                // deviatoric stress (sigma_xx, sigma_xy, sigma_yy) = (P_xx - p, P_xy, P_yy - p)
                double* o = out3 + 3 * (size_t)c;
                const double p = rho * ph.R * T;
                o[0] = (m[3] - rho * u * u) - p;
                o[1] = m[4] - rho * u * v;
                o[2] = (m[5] - rho * v * v) - p;
            }
            if (tot4) {
                const double V = geom[c].vol;
                double* o = tot4 + 4 * (size_t)c;
                o[0] = V * m[0]; o[1] = V * m[1]; o[2] = V * m[2]; o[3] = V * 0.5 * (m[3] + m[5] + m[8]);
            }
        }
    }
}

// Fixed-order sum of n rows of `width` doubles (one workgroup).
// Fixed-order sum of n rows of `width` (<= 4) doubles by one wavefront.
// Strict mode: the state of every cell from the raw moments of its stored
// g~, h~ (the chunk partials the update leaves, summed in chunk order), and a
// flag when a moment is not finite or rho or T is not positive.  rec[0] counts
// such cells, rec[1] holds the smallest such cell index (atomic min).
__global__ __launch_bounds__(BS) void k_check_state(const LevelDesc* __restrict__ lvs,
                                                    const int* __restrict__ cell_lev, int n_cells, Phys ph,
                                                    const double* __restrict__ cmom, int CH,
                                                    unsigned long long* __restrict__ rec) {
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n_cells; c += gridDim.x * blockDim.x) {
        double cm[NMOM];
        sum_chunks(cmom, c, n_cells, lvs[cell_lev[c]].N, CH, cm);
        bool bad = false;
        for (int k = 0; k < 11; ++k) bad = bad || !isfinite(cm[k]);
        double rho, u, v, T, qx, qy;
        raw_to_state(cm, cm[M_U0], cm[M_V0], ph, rho, u, v, T, qx, qy);
        bad = bad || !(rho > 0.0) || !(T > 0.0) || !isfinite(rho) || !isfinite(T) || !isfinite(u) || !isfinite(v);
        if (bad) {
            atomicAdd(rec, 1ull);
            atomicMin(rec + 1, (unsigned long long)c);
        }
    }
}

__global__ void k_sum_rows(const double* __restrict__ in, int n, int width, double* __restrict__ out) {
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int r = lane_id(); r < n; r += WL)
        for (int k = 0; k < width; ++k) v[k] += in[(size_t)r * width + k];
    wave_sum<4>(v);
    if (lane_id() == 0)
        for (int k = 0; k < width; ++k) out[k] = v[k];
}

// ---------------------------------------------------------------------------
// level switch: projection + four-moment mapping correction (Eq.
// level_switch_conservation), T_tar the cell temperature
// ---------------------------------------------------------------------------
template <typename S>
__global__ __launch_bounds__(BS) void k_remap(const LevelDesc* __restrict__ olv, const LevelDesc* __restrict__ nlv,
                                              const RemapItem* __restrict__ items, int n, Phys ph,
                                              unsigned long long* neg) {
    for (int it = item0(); it < n; it += istride()) {
        const RemapItem R = items[it];
        const LevelDesc& Ls = olv[R.src_lev];
        const LevelDesc& Ld = nlv[R.dst_lev];
        auto sg = rowp<S>(Ls.g, (size_t)R.src_slot * Ls.stride);
        auto sh = rowp<S>(Ls.h, (size_t)R.src_slot * Ls.stride);
        auto dg = rowp<S>(Ld.g, (size_t)R.dst_slot * Ld.stride);
        auto dh = rowp<S>(Ld.h, (size_t)R.dst_slot * Ld.stride);
        if (R.tab.off == nullptr) {
            for (int i = lane_id(); i < Ld.N; i += WL) { dg[i] = sg[i]; dh[i] = sh[i]; }
            continue;
        }
        double m[18];
#pragma unroll
        for (int k = 0; k < 18; ++k) m[k] = 0.0;
        for (int i = lane_id(); i < Ls.N; i += WL)
            acc_m9(m, gp(Ls.w)[i], gp(Ls.xi_x)[i], gp(Ls.xi_y)[i], (double)sg[i], (double)sh[i]);
        // Projection, RU destination points per lane at a time: their table
        // offsets, first entries and source values are loaded together (most
        // points have one entry: a refinement or an unchanged point), further
        // entries are added after in table order.
        constexpr int RU = 4;
        for (int P0 = lane_id(); P0 < Ld.N; P0 += WL * RU) {
            int e0[RU], e1[RU], a0[RU];
            double gP[RU], HP[RU];
#pragma unroll
            for (int q = 0; q < RU; ++q) {
                const int Pc = clampi(P0 + q * WL, Ld.N);
                e0[q] = gp(R.tab.off)[Pc];
                e1[q] = gp(R.tab.off)[Pc + 1];
            }
#pragma unroll
            for (int q = 0; q < RU; ++q) a0[q] = gp(R.tab.idx)[e0[q]];
#pragma unroll
            for (int q = 0; q < RU; ++q) {
                const int a = a0[q];
                const double fr = gp(R.tab.frac)[e0[q]];
                const double ga = (double)sg[a];
                const double xa = gp(Ls.xi_x)[a], ya = gp(Ls.xi_y)[a];
                gP[q] = 0.0;
                HP[q] = 0.0;
                gP[q] += fr * ga;
                HP[q] += fr * ((double)sh[a] + (xa * xa + ya * ya) * ga);
            }
#pragma unroll
            for (int q = 0; q < RU; ++q) {
                for (int e = e0[q] + 1; e < e1[q]; ++e) {
                    const int a = gp(R.tab.idx)[e];
                    const double fr = gp(R.tab.frac)[e];
                    const double ga = (double)sg[a];
                    const double xa = gp(Ls.xi_x)[a], ya = gp(Ls.xi_y)[a];
                    gP[q] += fr * ga;
                    HP[q] += fr * ((double)sh[a] + (xa * xa + ya * ya) * ga);
                }
                const int P = P0 + q * WL;
                if (P < Ld.N) {
                    const double x = gp(Ld.xi_x)[P], y = gp(Ld.xi_y)[P], w = gp(Ld.w)[P];
                    const S gs = (S)gP[q], hs = (S)(HP[q] - (x * x + y * y) * gP[q]);
                    dg[P] = gs;
                    dh[P] = hs;
                    acc_m9(m + 9, w, x, y, (double)gs, (double)hs);
                }
            }
        }
        wave_sum<18>(m);
        int nf = 0;
        if (ph.map_moments) {
            const double rho = m[0], u = m[1] / rho, v = m[2] / rho;
            const double T = (2.0 * m[3] / rho - (u * u + v * v)) / ((3.0 + ph.K) * ph.R);
            double dM[9];
            for (int k = 0; k < 9; ++k) dM[k] = m[k] - m[9 + k];
            map_correct_apply<S>(Ld, dg, dh, dM, m, T, ph, nf, neg);
        }
        nf = __any(nf);
        if (lane_id() == 0 && nf) atomicAdd(neg, 1ull);
    }
}

// ---------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------
// Workgroups for n items at `per` items each, in whole rounds over the XCDs
// (see wg_index).
static inline int grid_for(int n, int per = MAXW) {
    int b = (n + per - 1) / per;
    b = (b + NXCD - 1) / NXCD * NXCD;
    return b < NXCD ? NXCD : (b > 1048576 ? 1048576 : b);
}

// Tunable kernels are instantiated for several (points per lane per chunk U,
// minimum waves per SIMD) pairs; the variant index selects one at launch.
// (1, 2) gives the FP64 fused kernels 256 VGPRs, where (1, 4) spills.
constexpr int N_VARIANTS = 5;
#define MLVS_LAUNCH_UW(prec, KERNEL, U_, W_, ...)                                                \
    do {                                                                                        \
        if ((prec) == 32) hipLaunchKernelGGL((KERNEL<float, U_, W_>), __VA_ARGS__);              \
        else hipLaunchKernelGGL((KERNEL<double, U_, W_>), __VA_ARGS__);                          \
    } while (0)
#define MLVS_DISPATCH_V(prec, var, KERNEL, ...)                                                  \
    do {                                                                                        \
        switch (var) {                                                                          \
        case 0: MLVS_LAUNCH_UW(prec, KERNEL, 1, 4, __VA_ARGS__); break;                          \
        case 2: MLVS_LAUNCH_UW(prec, KERNEL, 4, 2, __VA_ARGS__); break;                          \
        case 3: MLVS_LAUNCH_UW(prec, KERNEL, 4, 4, __VA_ARGS__); break;                          \
        case 4: MLVS_LAUNCH_UW(prec, KERNEL, 1, 2, __VA_ARGS__); break;                          \
        default: MLVS_LAUNCH_UW(prec, KERNEL, 2, 4, __VA_ARGS__); break;                         \
        }                                                                                       \
    } while (0)

#define MLVS_LAUNCH_UWC(prec, KERNEL, U_, W_, C_, ...)                                           \
    do {                                                                                        \
        if ((prec) == 32) hipLaunchKernelGGL((KERNEL<float, U_, W_, C_>), __VA_ARGS__);          \
        else hipLaunchKernelGGL((KERNEL<double, U_, W_, C_>), __VA_ARGS__);                      \
    } while (0)
#define MLVS_DISPATCH_VC1(prec, var, C_, KERNEL, ...)                                            \
    do {                                                                                        \
        switch (var) {                                                                          \
        case 0: MLVS_LAUNCH_UWC(prec, KERNEL, 1, 4, C_, __VA_ARGS__); break;                     \
        case 2: MLVS_LAUNCH_UWC(prec, KERNEL, 4, 2, C_, __VA_ARGS__); break;                     \
        case 3: MLVS_LAUNCH_UWC(prec, KERNEL, 4, 4, C_, __VA_ARGS__); break;                     \
        case 4: MLVS_LAUNCH_UWC(prec, KERNEL, 1, 2, C_, __VA_ARGS__); break;                     \
        default: MLVS_LAUNCH_UWC(prec, KERNEL, 2, 4, C_, __VA_ARGS__); break;                    \
        }                                                                                       \
    } while (0)
// ... and for the kernels instantiated per compatibility order (4 or 8 moments)
#define MLVS_DISPATCH_VC(prec, var, cm, KERNEL, ...)                                             \
    do {                                                                                        \
        if ((cm) == 8) MLVS_DISPATCH_VC1(prec, var, 8, KERNEL, __VA_ARGS__);                     \
        else MLVS_DISPATCH_VC1(prec, var, 4, KERNEL, __VA_ARGS__);                               \
    } while (0)

// ... and per mesh kind (unstructured meshes: the (1, 4) pair for every
// variant; with two points per lane the larger limiter stencil spills)
#define MLVS_LAUNCH_UWM(prec, KERNEL, U_, W_, M_, ...)                                           \
    do {                                                                                        \
        if ((prec) == 32) hipLaunchKernelGGL((KERNEL<float, U_, W_, M_>), __VA_ARGS__);          \
        else hipLaunchKernelGGL((KERNEL<double, U_, W_, M_>), __VA_ARGS__);                      \
    } while (0)
#define MLVS_DISPATCH_VM(prec, var, mk, KERNEL, ...)                                             \
    do {                                                                                        \
        if (mk) {                                                                               \
            MLVS_LAUNCH_UWM(prec, KERNEL, 1, 4, 1, __VA_ARGS__);                                 \
        } else {                                                                                \
            switch (var) {                                                                      \
            case 0: MLVS_LAUNCH_UWM(prec, KERNEL, 1, 4, 0, __VA_ARGS__); break;                  \
            case 2: MLVS_LAUNCH_UWM(prec, KERNEL, 4, 2, 0, __VA_ARGS__); break;                  \
            case 3: MLVS_LAUNCH_UWM(prec, KERNEL, 4, 4, 0, __VA_ARGS__); break;                  \
            case 4: MLVS_LAUNCH_UWM(prec, KERNEL, 1, 2, 0, __VA_ARGS__); break;                  \
            default: MLVS_LAUNCH_UWM(prec, KERNEL, 2, 4, 0, __VA_ARGS__); break;                 \
            }                                                                                   \
        }                                                                                       \
    } while (0)
#define MLVS_LAUNCH_UWCM(prec, KERNEL, U_, W_, C_, M_, ...)                                      \
    do {                                                                                        \
        if ((prec) == 32) hipLaunchKernelGGL((KERNEL<float, U_, W_, C_, M_>), __VA_ARGS__);      \
        else hipLaunchKernelGGL((KERNEL<double, U_, W_, C_, M_>), __VA_ARGS__);                  \
    } while (0)
#define MLVS_DISPATCH_VCM1(prec, var, C_, mk, KERNEL, ...)                                       \
    do {                                                                                        \
        if (mk) {                                                                               \
            MLVS_LAUNCH_UWCM(prec, KERNEL, 1, 4, C_, 1, __VA_ARGS__);                            \
        } else {                                                                                \
            switch (var) {                                                                      \
            case 0: MLVS_LAUNCH_UWCM(prec, KERNEL, 1, 4, C_, 0, __VA_ARGS__); break;             \
            case 2: MLVS_LAUNCH_UWCM(prec, KERNEL, 4, 2, C_, 0, __VA_ARGS__); break;             \
            case 3: MLVS_LAUNCH_UWCM(prec, KERNEL, 4, 4, C_, 0, __VA_ARGS__); break;             \
            case 4: MLVS_LAUNCH_UWCM(prec, KERNEL, 1, 2, C_, 0, __VA_ARGS__); break;             \
            default: MLVS_LAUNCH_UWCM(prec, KERNEL, 2, 4, C_, 0, __VA_ARGS__); break;            \
            }                                                                                   \
        }                                                                                       \
    } while (0)
#define MLVS_DISPATCH_VCM(prec, var, cm, mk, KERNEL, ...)                                        \
    do {                                                                                        \
        if ((cm) == 8) MLVS_DISPATCH_VCM1(prec, var, 8, mk, KERNEL, __VA_ARGS__);                \
        else MLVS_DISPATCH_VCM1(prec, var, 4, mk, KERNEL, __VA_ARGS__);                          \
    } while (0)

int variant_count() { return N_VARIANTS; }

#define MLVS_DISPATCH(prec, KERNEL, ...)                                                        \
    do {                                                                                        \
        if ((prec) == 32) hipLaunchKernelGGL(KERNEL<float>, __VA_ARGS__);                        \
        else hipLaunchKernelGGL(KERNEL<double>, __VA_ARGS__);                                    \
    } while (0)

hipError_t launch_cell_prep(int prec, hipStream_t st, const LevelDesc* lv, const int* cell_lev, const int* cell_slot,
                            const int* order, int n_cells, Phys ph, double* params, const double* cmom, int CH,
                            int var) {
    if (n_cells <= 0) return hipSuccess;
    MLVS_DISPATCH_VC(prec, var, ph.compat, k_cell_prep, dim3(grid_for(n_cells, GW)), dim3(GBS), 0, st, lv, cell_lev,
                     cell_slot, order, n_cells, ph, params, cmom, CH);
    return hipGetLastError();
}

hipError_t launch_raw_moments(int prec, hipStream_t st, const LevelDesc* lv, const int* cell_lev,
                              const int* cell_slot, int n_cells, const double* params, double* cmom, int CH,
                              int nch) {
    if (n_cells <= 0) return hipSuccess;
    MLVS_DISPATCH(prec, k_raw_moments, dim3(grid_for(n_cells * nch)), dim3(BS), 0, st, lv, cell_lev, cell_slot,
                  n_cells, params, cmom, CH, nch);
    return hipGetLastError();
}

hipError_t launch_init_eq(int prec, hipStream_t st, const LevelDesc* lv, const int* cell_lev, const int* cell_slot,
                          int n_cells, const double* rho_u_v_T, Phys ph, double* params) {
    if (n_cells <= 0) return hipSuccess;
    MLVS_DISPATCH(prec, k_init_eq, dim3(grid_for(n_cells)), dim3(BS), 0, st, lv, cell_lev, cell_slot, n_cells,
                  rho_u_v_T, ph, params);
    return hipGetLastError();
}

hipError_t launch_ghost(int prec, hipStream_t st, const LevelDesc* lv, const GhostItem* items, int n,
                        const int* cell_lev, const int* cell_slot, const double* params, Phys ph,
                        unsigned long long* neg) {
    if (n <= 0) return hipSuccess;
    MLVS_DISPATCH(prec, k_ghost, dim3(grid_for(n)), dim3(BS), 0, st, lv, items, n, cell_lev, cell_slot, params, ph,
                  neg);
    return hipGetLastError();
}

hipError_t launch_face_rec(int prec, hipStream_t st, const LevelDesc* lv, const FaceItem* items, int n,
                           const int* cell_slot, const int* cell_nbr, const CellGeom* geom, const double* params,
                           Phys ph, double* fmom, int CH, int nch, int var) {
    if (n <= 0) return hipSuccess;
    MLVS_DISPATCH_VM(prec, var, ph.mesh_kind, k_face_rec, dim3(grid_for(n * nch)), dim3(BS), 0, st, lv, items, n,
                     cell_slot, cell_nbr, geom, params, ph, fmom, CH, nch);
    return hipGetLastError();
}

hipError_t launch_face_target(int prec, hipStream_t st, const LevelDesc* lv, const FaceItem* items, int n,
                              const BCDev* bcs, Phys ph, const double* fmom, double* fpar, int CH, int var) {
    if (n <= 0) return hipSuccess;
    MLVS_DISPATCH_VC(prec, var, ph.compat, k_face_target, dim3(grid_for(n, GW)), dim3(GBS), 0, st, lv, items, n, bcs,
                     ph, fmom, fpar, CH);
    return hipGetLastError();
}

hipError_t launch_face_full(int prec, hipStream_t st, const LevelDesc* lv, const FaceItem* items, int n,
                            const int* cell_slot, const int* cell_nbr, const CellGeom* geom, const double* params,
                            const BCDev* bcs, Phys ph, double* fpar, int var) {
    if (n <= 0) return hipSuccess;
    MLVS_DISPATCH_VCM(prec, var, ph.compat, ph.mesh_kind, k_face_full, dim3(grid_for(n)), dim3(BS), 0, st, lv, items,
                      n, cell_slot, cell_nbr, geom, params, bcs, ph, fpar);
    return hipGetLastError();
}

hipError_t launch_update_cell(int prec, hipStream_t st, const LevelDesc* lv, const int* cell_lev,
                              const int* cell_slot, const int* order, int n_cells, const CellGeom* geom,
                              const int* cell_frow, const FaceItem* items, const double* fpar, double* params,
                              Phys ph, double* cmom, int var) {
    if (n_cells <= 0) return hipSuccess;
    MLVS_DISPATCH_VC(prec, var, ph.compat, k_update_cell, dim3(grid_for(n_cells)), dim3(BS), 0, st, lv, cell_lev,
                     cell_slot, order, n_cells, geom, cell_frow, items, fpar, params, ph, cmom);
    return hipGetLastError();
}

hipError_t launch_update(int prec, hipStream_t st, const LevelDesc* lv, const int* cell_lev, const int* cell_slot,
                         const int* order, int n_cells, const CellGeom* geom, const int* cell_frow,
                         const FaceItem* items, const double* fpar, const double* params, Phys ph, double* cmom,
                         int CH, int nch, int var) {
    if (n_cells <= 0) return hipSuccess;
    MLVS_DISPATCH_V(prec, var, k_update, dim3(grid_for(n_cells * nch)), dim3(BS), 0, st, lv, cell_lev, cell_slot,
                    order, n_cells, geom, cell_frow, items, fpar, params, ph, cmom, CH, nch);
    return hipGetLastError();
}

hipError_t launch_cell_moments(int prec, hipStream_t st, const LevelDesc* lv, const int* cell_lev,
                               const int* cell_slot, int n_cells, const CellGeom* geom, Phys ph, double* out6,
                               double* tot4, double* out8, double* out3) {
    if (n_cells <= 0) return hipSuccess;
    MLVS_DISPATCH(prec, k_cell_moments, dim3(grid_for(n_cells)), dim3(BS), 0, st, lv, cell_lev, cell_slot, n_cells,
                  geom, ph, out6, tot4, out8, out3);
    return hipGetLastError();
}

hipError_t launch_check_state(hipStream_t st, const LevelDesc* lv, const int* cell_lev, int n_cells, Phys ph,
                              const double* cmom, int CH, unsigned long long* rec) {
    if (n_cells <= 0) return hipSuccess;
    const int blocks = (n_cells + BS - 1) / BS;
    k_check_state<<<blocks < 65535 ? blocks : 65535, BS, 0, st>>>(lv, cell_lev, n_cells, ph, cmom, CH, rec);
    return hipGetLastError();
}

hipError_t launch_sum_rows(hipStream_t st, const double* in, int n, int width, double* out) {
    hipLaunchKernelGGL(k_sum_rows, dim3(1), dim3(WL), 0, st, in, n, width, out);
    return hipGetLastError();
}

hipError_t launch_remap(int prec, hipStream_t st, const LevelDesc* old_lv, const LevelDesc* new_lv,
                        const RemapItem* items, int n, Phys ph, unsigned long long* neg) {
    if (n <= 0) return hipSuccess;
    MLVS_DISPATCH(prec, k_remap, dim3(grid_for(n)), dim3(BS), 0, st, old_lv, new_lv, items, n, ph, neg);
    return hipGetLastError();
}


// ---------------------------------------------------------------------------
// cross-level faces (Sec. 3.4): states refined to V_int = min(kappa_L, kappa_R)
// and corrected to their own native moments (Eq. interface_state_moment_matching),
// slopes refined by inheritance, DUGKS face evaluation on V_int, the interface
// microflux (Eq. interface_reduced_fluxes) coarsened to each native level and
// corrected to the common target F_int (Eq. native_flux_moment_matching).
// ---------------------------------------------------------------------------

// phi_bar+ and slope of one side at interface point P (parent a on the native level).
template <typename S, typename SD>
__device__ __forceinline__ void side_refined(const SD& sd, const LevelDesc& Ln, const LevelDesc& LI, int a,
                                             int P, S (&f)[2], S (&sx)[2], S (&sy)[2]) {
    side_slope<S>(sd, a, f, sx, sy);
    const double xa = gp(Ln.xi_x)[a], ya = gp(Ln.xi_y)[a], xP = gp(LI.xi_x)[P], yP = gp(LI.xi_y)[P];
    const S dq = (S)((xa * xa + ya * ya) - (xP * xP + yP * yP));
    f[1] = f[1] + dq * f[0];
    sx[1] = sx[1] + dq * sx[0];
    sy[1] = sy[1] + dq * sy[0];
}

template <typename S, int U, int MK>
__device__ __forceinline__ void xface_items(const LevelDesc* __restrict__ lvs, const XFaceItem* __restrict__ items,
                                            int n, const int* __restrict__ cell_slot,
                                            const int* __restrict__ cell_nbr, const CellGeom* __restrict__ geom,
                                            const double* __restrict__ params, Phys ph, unsigned long long* neg,
                                            int first, int stride) {
    const S s = (S)(0.5 * ph.dt);
    for (int it = first; it < n; it += stride) {
        const XFaceItem F = items[it];
        const LevelDesc& LA = lvs[F.levA];
        const LevelDesc& LB = lvs[F.levB];
        const LevelDesc& LI = lvs[F.levI];
        SideOf<S, MK> sL, sR;
        load_side<S>(sL, LA, F.L, cell_slot, cell_nbr, geom, F.dLx, F.dLy);
        load_side<S>(sR, LB, F.R, cell_slot, cell_nbr, geom, F.dRx, F.dRy);
        const double TL = params[(size_t)F.L * NPARAM + P_T], TR = params[(size_t)F.R * NPARAM + P_T];
        // pass 1: provisional refined states and native target moments
        double m[36];
#pragma unroll
        for (int k = 0; k < 36; ++k) m[k] = 0.0;
        for (int P = lane_id(); P < LI.N; P += WL) {
            const double x = gp(LI.xi_x)[P], y = gp(LI.xi_y)[P], w = gp(LI.w)[P];
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                const SideOf<S, MK>& sd = side ? sR : sL;
                const LevelDesc& Ln = side ? LB : LA;
                const PairTable& tb = side ? F.IfromB : F.IfromA;
                const int a = gp(tb.idx)[gp(tb.off)[P]];
                S f[2], sx[2], sy[2];
                side_slope<S>(sd, a, f, sx, sy);
                const double xa = gp(Ln.xi_x)[a], ya = gp(Ln.xi_y)[a];
                const double ga = (double)f[0], ha = (double)f[1];
                const double hP = ha + ((xa * xa + ya * ya) - (x * x + y * y)) * ga;
                double* mm = m + 18 * side;
                acc_m9(mm, w, x, y, ga, hP);          // provisional, on V_int
                acc_m9(mm + 9, w, xa, ya, ga, ha);    // native (the parent's weight is the children's sum)
            }
        }
        wave_sum<36>(m);
        MapCoef cL{}, cR{};
        if (ph.map_moments) {
            for (int side = 0; side < 2; ++side) {
                const double* mm = m + 18 * side;
                double dM[9];
                for (int k = 0; k < 9; ++k) dM[k] = mm[9 + k] - mm[k];
                (side ? cR : cL) = map_coeffs(LI, dM, side ? TR : TL, ph);
            }
        }
        const double u0 = 0.5 * (params[(size_t)F.L * NPARAM + P_U] + params[(size_t)F.R * NPARAM + P_U]);
        const double v0 = 0.5 * (params[(size_t)F.L * NPARAM + P_V] + params[(size_t)F.R * NPARAM + P_V]);
        auto rg = rowp<S>(LI.Fg, (size_t)F.scratch * LI.stride);
        auto rh = rowp<S>(LI.Fh, (size_t)F.scratch * LI.stride);
        // pass 2: corrected states, upwind reconstruction on V_int, face moments
        double fm[11];
#pragma unroll
        for (int k = 0; k < 11; ++k) fm[k] = 0.0;
        int nf = 0;
        for (int P = lane_id(); P < LI.N; P += WL) {
            const double xd = gp(LI.xi_x)[P], yd = gp(LI.xi_y)[P];
            const S x = (S)xd, y = (S)yd;
            S e[2][2];
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                const SideOf<S, MK>& sd = side ? sR : sL;
                const LevelDesc& Ln = side ? LB : LA;
                const PairTable& tb = side ? F.IfromB : F.IfromA;
                const int a = gp(tb.idx)[gp(tb.off)[P]];
                S f[2], sx[2], sy[2];
                side_refined<S>(sd, Ln, LI, a, P, f, sx, sy);
                double dg, dh;
                map_delta(side ? cR : cL, xd, yd, dg, dh);
                const S gprov = f[0];
                f[0] = (S)((double)f[0] + dg);
                f[1] = (S)((double)f[1] + dh);
                if (f[0] < S(0) && gprov >= S(0)) nf = 1;
                e[side][0] = f[0] + ((S)sd.dx - x * s) * sx[0] + ((S)sd.dy - y * s) * sy[0];
                e[side][1] = f[1] + ((S)sd.dx - x * s) * sx[1] + ((S)sd.dy - y * s) * sy[1];
            }
            const double dn = xd * F.nx + yd * F.ny;
            S eg, eh;
            if (dn > 0) { eg = e[0][0]; eh = e[0][1]; }
            else if (dn < 0) { eg = e[1][0]; eh = e[1][1]; }
            else { eg = S(0.5) * (e[0][0] + e[1][0]); eh = S(0.5) * (e[0][1] + e[1][1]); }
            rg[P] = eg;
            rh[P] = eh;
            acc_raw<S>(fm, gp(LI.w)[P], xd - u0, yd - v0, eg, eh);
        }
        wave_sum<11>(fm);
        double c1, c2;
        double Tf = 1.0;
        const Eq<S> eq = eq_cast<S>(face_target<S, 1>(LI, fm, u0, v0, ph, ph.compat && ph.face_compat, c1, c2, &Tf));
        // pass 3: interface microflux per unit area and its moments F_int
        double Fm[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) Fm[k] = 0.0;
        const S k1 = (S)c1, k2 = (S)c2;
        for (int P = lane_id(); P < LI.N; P += WL) {
            const double xd = gp(LI.xi_x)[P], yd = gp(LI.xi_y)[P], w = gp(LI.w)[P];
            S gs, hs;
            eq_eval<S>(eq, (S)xd, (S)yd, gs, hs);
            const S dn = (S)(xd * F.nx + yd * F.ny);
            const S fg = dn * (k1 * rg[P] + k2 * gs);
            const S fh = dn * (k1 * rh[P] + k2 * hs);
            rg[P] = fg;
            rh[P] = fh;
            acc_m9(Fm, w, xd, yd, (double)fg, (double)fh);
        }
        wave_sum<9>(Fm);
        __threadfence_block();   // pass 4 reads interface rows written by other lanes
        // pass 4: coarsen to both native levels (provisional) and their moments
        double pm[18];
#pragma unroll
        for (int k = 0; k < 18; ++k) pm[k] = 0.0;
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const LevelDesc& Ln = side ? LB : LA;
            const PairTable& tb = side ? F.BfromI : F.AfromI;
            auto og = rowp<S>(Ln.Fg, (size_t)(side ? F.rowB : F.rowA) * Ln.stride);
            auto oh = rowp<S>(Ln.Fh, (size_t)(side ? F.rowB : F.rowA) * Ln.stride);
            for (int a = lane_id(); a < Ln.N; a += WL) {
                double gA = 0.0, HA = 0.0;
                for (int e = gp(tb.off)[a]; e < gp(tb.off)[a + 1]; ++e) {
                    const int P = gp(tb.idx)[e];
                    const double fr = gp(tb.frac)[e];
                    const double xP = gp(LI.xi_x)[P], yP = gp(LI.xi_y)[P];
                    const double gP = (double)rg[P];
                    gA += fr * gP;
                    HA += fr * ((double)rh[P] + (xP * xP + yP * yP) * gP);
                }
                const double x = gp(Ln.xi_x)[a], y = gp(Ln.xi_y)[a], w = gp(Ln.w)[a];
                const S gs = (S)gA, hs = (S)(HA - (x * x + y * y) * gA);
                og[a] = gs;
                oh[a] = hs;
                acc_m9(pm + 9 * side, w, x, y, (double)gs, (double)hs);
            }
        }
        wave_sum<18>(pm);
        // pass 5: flux correction to F_int (T_tar = face T for four moments), times area
        const S ar = (S)F.area;
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const LevelDesc& Ln = side ? LB : LA;
            auto og = rowp<S>(Ln.Fg, (size_t)(side ? F.rowB : F.rowA) * Ln.stride);
            auto oh = rowp<S>(Ln.Fh, (size_t)(side ? F.rowB : F.rowA) * Ln.stride);
            MapCoef mc{};
            if (ph.map_moments) {
                double dM[9];
                for (int k = 0; k < 9; ++k) dM[k] = Fm[k] - pm[9 * side + k];
                mc = map_coeffs(Ln, dM, Tf, ph);
            }
            for (int a = lane_id(); a < Ln.N; a += WL) {
                const double x = gp(Ln.xi_x)[a], y = gp(Ln.xi_y)[a];
                double dg, dh;
                map_delta(mc, x, y, dg, dh);
                og[a] = ar * (S)((double)og[a] + dg);
                oh[a] = ar * (S)((double)oh[a] + dh);
            }
        }
        nf = __any(nf);
        if (lane_id() == 0 && nf) atomicAdd(neg, 1ull);
    }
}

template <typename S, int U, int MINW, int MK>
__global__ __launch_bounds__(BS, MINW) void k_xface(const LevelDesc* __restrict__ lvs, const XFaceItem* __restrict__ items,
                                              int n, const int* __restrict__ cell_slot,
                                              const int* __restrict__ cell_nbr, const CellGeom* __restrict__ geom,
                                              const double* __restrict__ params, Phys ph, unsigned long long* neg) {
    xface_items<S, U, MK>(lvs, items, n, cell_slot, cell_nbr, geom, params, ph, neg, item0(), istride());
}

// ---------------------------------------------------------------------------
// criterion (Sec. 3.2): per cell, on the stored distribution refined to V_base
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// The tensor base grid's axes (x, wx, y, wy), staged in LDS by the criterion
// kernel when each axis has at most CRIT_AXIS nodes: the block tests then read
// node coordinates and weights from LDS instead of per-point arrays (their
// scattered per-lane reads made the address unit the bottleneck).
constexpr int CRIT_AXIS = 512;
__shared__ double crit_axes[4 * CRIT_AXIS];

// Inheritance (Sec. 3.3.2) gives every base point under a level point p the
// level point's g and H = h + |xi_p|^2 g.  Every sum the criterion takes over
// a block of V_base therefore splits into g_p, H_p times sums that depend on
// the base grid alone: over a block inside one level point, the block's own
// tables (ctab); over a block the level splits, the sum of its parts, down to
// single base points.  A cell's row is read once; nothing is expanded to
// V_base.
//
// Base-grid tables per aligned block (scales 1, 2, 3 one after another):
// W = sum w, the velocity centroid (sum w xi_x, sum w xi_y) / W, P[d][s] =
// sum_{s xi_d >= 0} w xi_d, Q[d][s][e] = sum_{s xi_d >= 0} w xi_d xi_e
// (s = 0: +, 1: -).
enum { CT_W = 0, CT_WX = 1, CT_WY = 2, CT_P = 3, CT_Q = 7, NCT = 15 };
// Level-point tables: |xi_p|^2, then over the point's base members sum w|x|,
// sum w|y|, sum w x^2, sum w|x y|, sum w y^2 (the normalisations S_r).
enum { PT_X2 = 0, PT_AX = 1, PT_AY = 2, PT_BXX = 3, PT_BXY = 4, PT_BYY = 5, NPT = 6 };

struct CritCtx {
    bool axes_lds;            // crit_axes holds the axes
    const double* axes;       // x [nx], wx [nx], y [ny], wy [ny] (global)
    const int* ptb;           // base -> level point of the cell's level
    const double* ptab;       // level-point tables of the cell's level [N][NPT]
    const uint8_t* klev;      // kappa of the cell's current level
    const double *T1, *T2, *T3;   // base-grid block tables of scales 1, 2, 3
    int nx, ny, nbx, n4x, n8x;
    double merge_rho, merge_E, split_rho, split_E;   // C_merge rho_tot, C_merge E_tot, C_split ...
    double epsS[4];                                  // eps_merge S_r
    int flux_test;
};

// Sums of one block: sum w g, sum w H, and the half-range fluxes
// F[r][d][s] = sum_{s xi_d >= 0} w xi_d m_r, m = (g, xi_x g, xi_y g, H/2).
struct CritAcc {
    double m1, mH, F[4][2][2];
};

__device__ __forceinline__ void acc_zero(CritAcc& a) {
    a.m1 = 0.0;
    a.mH = 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int d = 0; d < 2; ++d) { a.F[r][d][0] = 0.0; a.F[r][d][1] = 0.0; }
}

// A block inside one level point: g and H times the block's tables (FULL:
// also the half-range fluxes).
template <bool FULL>
__device__ __forceinline__ void acc_table(CritAcc& a, double gv, double Hv, const double* T) {
    a.m1 += gv * T[CT_W];
    a.mH += Hv * T[CT_W];
    if (!FULL) return;
#pragma unroll
    for (int d = 0; d < 2; ++d)
#pragma unroll
        for (int sg = 0; sg < 2; ++sg) {
            const double P = T[CT_P + 2 * d + sg];
            a.F[0][d][sg] += gv * P;
            a.F[1][d][sg] += gv * T[CT_Q + 4 * d + 2 * sg];
            a.F[2][d][sg] += gv * T[CT_Q + 4 * d + 2 * sg + 1];
            a.F[3][d][sg] += 0.5 * Hv * P;
        }
}

// One base point (ix, iy) carrying g and H.
template <bool FULL>
__device__ __forceinline__ void acc_base(CritAcc& a, const CritCtx& cc, double gv, double Hv, int ix, int iy) {
    double w, x, y;
    if (cc.axes_lds) {
        x = crit_axes[ix];
        y = crit_axes[2 * CRIT_AXIS + iy];
        w = crit_axes[CRIT_AXIS + ix] * crit_axes[3 * CRIT_AXIS + iy];
    } else {
        x = cc.axes[ix];
        y = cc.axes[2 * cc.nx + iy];
        w = cc.axes[cc.nx + ix] * cc.axes[2 * cc.nx + cc.ny + iy];
    }
    a.m1 += w * gv;
    a.mH += w * Hv;
    if (!FULL) return;
    const double xd[2] = {x, y};
    const double mr[4] = {gv, x * gv, y * gv, 0.5 * Hv};
#pragma unroll
    for (int d = 0; d < 2; ++d) {
        // w xi_d on the point's half-range (a point with xi_d = 0 adds zero to both)
        const double t = w * xd[d];
        const double tp = xd[d] >= 0 ? t : 0.0, tn = xd[d] >= 0 ? 0.0 : t;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            a.F[r][d][0] += tp * mr[r];
            a.F[r][d][1] += tn * mr[r];
        }
    }
}

template <typename S>
__device__ __forceinline__ void crit_gh(const CritCtx& cc, gptr<S> g, gptr<S> h, int b, double& gv, double& Hv) {
    const int p = cc.ptb[b];
    gv = (double)g[p];
    Hv = (double)h[p] + cc.ptab[(size_t)p * NPT + PT_X2] * gv;
}

template <typename S, bool FULL>
__device__ __forceinline__ void crit_sum2(CritAcc& a, const CritCtx& cc, gptr<S> g, gptr<S> h, int X, int Y) {
    // every load of the block is issued before its value is needed (the
    // level's mask decides afterwards whether the block is one point or four):
    // two dependent load steps instead of three
    const int b0 = 2 * X + cc.nx * 2 * Y;
    const int kb = cc.klev[X + cc.nbx * Y];
    int p[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) p[q] = cc.ptb[b0 + (q & 1) + cc.nx * (q >> 1)];
    double gv[4], Hv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        gv[q] = (double)g[p[q]];
        Hv[q] = (double)h[p[q]] + cc.ptab[(size_t)p[q] * NPT + PT_X2] * gv[q];
    }
    if (kb >= 1) {
        acc_table<FULL>(a, gv[0], Hv[0], cc.T1 + (size_t)(X + cc.nbx * Y) * NCT);
        return;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) acc_base<FULL>(a, cc, gv[q], Hv[q], 2 * X + (q & 1), 2 * Y + (q >> 1));
}

template <typename S, bool FULL>
__device__ __forceinline__ void crit_sum4(CritAcc& a, const CritCtx& cc, gptr<S> g, gptr<S> h, int X, int Y) {
    if (cc.klev[2 * X + cc.nbx * 2 * Y] >= 2) {
        double gv, Hv;
        crit_gh<S>(cc, g, h, 4 * X + cc.nx * 4 * Y, gv, Hv);
        acc_table<FULL>(a, gv, Hv, cc.T2 + (size_t)(X + cc.n4x * Y) * NCT);
        return;
    }
    for (int k = 0; k < 4; ++k) crit_sum2<S, FULL>(a, cc, g, h, 2 * X + (k & 1), 2 * Y + (k >> 1));
}

template <typename S, bool FULL>
__device__ __forceinline__ void crit_sum8(CritAcc& a, const CritCtx& cc, gptr<S> g, gptr<S> h, int X, int Y) {
    if (cc.klev[4 * X + cc.nbx * 4 * Y] >= 3) {
        double gv, Hv;
        crit_gh<S>(cc, g, h, 8 * X + cc.nx * 8 * Y, gv, Hv);
        acc_table<FULL>(a, gv, Hv, cc.T3 + (size_t)(X + cc.n8x * Y) * NCT);
        return;
    }
    for (int k = 0; k < 4; ++k) crit_sum4<S, FULL>(a, cc, g, h, 2 * X + (k & 1), 2 * Y + (k >> 1));
}

template <typename S, bool FULL>
__device__ __forceinline__ void crit_sum(CritAcc& a, const CritCtx& cc, gptr<S> g, gptr<S> h, int s, int X, int Y) {
    acc_zero(a);
    if (s == 3) crit_sum8<S, FULL>(a, cc, g, h, X, Y);
    else if (s == 2) crit_sum4<S, FULL>(a, cc, g, h, X, Y);
    else crit_sum2<S, FULL>(a, cc, g, h, X, Y);
}

// The transport-error test of Eqs. merge-transport-error and
// combined-merge-condition for a block with full sums a and tables T:
// max_r |F_fine - F_merged| / S_r <= eps_merge, evaluated as |F_fine -
// F_merged| <= eps_merge S_r.  The merged point (w_B, xi_B, g_B, H_B) gives
// F_merged = w_B xi_B,d m_r(B) = xi_B,d (m1, xi_B,x m1, xi_B,y m1, mH/2) on
// its half-range, with m1 = sum w g and mH = sum w H of the block.
__device__ __forceinline__ bool crit_flux_ok(const CritCtx& cc, const CritAcc& a, const double* T) {
    const double xB = T[CT_WX], yB = T[CT_WY];      // the block's velocity centroid
    const double mB[4] = {a.m1, xB * a.m1, yB * a.m1, 0.5 * a.mH};
    const double xdB[2] = {xB, yB};
    bool ok = true;
#pragma unroll
    for (int d = 0; d < 2; ++d)
#pragma unroll
        for (int sg = 0; sg < 2; ++sg) {
            const bool on = (sg == 0) ? (xdB[d] >= 0) : (-xdB[d] >= 0);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const double Fm = on ? xdB[d] * mB[r] : 0.0;
                ok = ok && fabs(a.F[r][d][sg] - Fm) <= cc.epsS[r];
            }
        }
    return ok;
}

// The indicator part of the merge test (Eqs. block-contribution-indicator,
// block-hysteresis-rule) from the block's mass and energy sums:
// I = max(m1 / rho_tot, mH / (2 E_tot)) against C_merge and C_split, as
// products with the totals; prev_merged holds when the cell's current level
// merges the block (for a consistent mask, when its first 2x2 child c2 has
// kappa >= s).
__device__ __forceinline__ bool crit_candidate(const CritCtx& cc, double m1, double mH, int s, int c2) {
    const double e = 0.5 * mH;
    const bool below_merge = m1 < cc.merge_rho && e < cc.merge_E;
    const bool below_split = m1 <= cc.split_rho && e <= cc.split_E;
    const bool prev_merged = cc.klev[c2] >= s;
    return below_merge || (below_split && prev_merged);
}

// The whole merge test of one block, summed from the level's points (the
// top-level blocks outside the 8x8 lattice).  The sixteen half-range fluxes
// are summed in a second pass, for candidates only.
template <typename S>
__device__ __forceinline__ bool crit_test(const CritCtx& cc, gptr<S> g, gptr<S> h, int s, int X, int Y) {
    const double* T = (s == 3 ? cc.T3 + (size_t)(X + cc.n8x * Y) * NCT
                       : s == 2 ? cc.T2 + (size_t)(X + cc.n4x * Y) * NCT : cc.T1 + (size_t)(X + cc.nbx * Y) * NCT);
    const int c2 = (X << (s - 1)) + cc.nbx * (Y << (s - 1));
    CritAcc a;
    crit_sum<S, false>(a, cc, g, h, s, X, Y);
    bool cand = crit_candidate(cc, a.m1, a.mH, s, c2);
    if (cand && cc.flux_test) {
        crit_sum<S, true>(a, cc, g, h, s, X, Y);
        cand = crit_flux_ok(cc, a, T);
    }
    return cand;
}

// Sum of a value over the four lanes of an aligned group of four, as
// (v0 + v1) + (v2 + v3) on all four lanes, by two quad exchanges: lanes 4j,
// 4j+1 form v0 + v1 and lanes 4j+2, 4j+3 form v2 + v3 (each pair the same
// value, addition being commutative), then every lane adds the other pair's
// sum.  The four lanes of a group always run together, so every source lane
// is active.
__device__ __forceinline__ double group4_sum(double v) {
    const double x = v + dpp_mov<0xB1>(v);       // quad_perm [1,0,3,2]
    return x + dpp_mov<0x4E>(x);                 // quad_perm [2,3,0,1]
}

template <typename S>
__global__ __launch_bounds__(BS, 2) void k_criterion(const LevelDesc* __restrict__ lvs, const int* __restrict__ cell_lev,
                                                  const int* __restrict__ cell_slot, int n_cells,
                                                  const int* __restrict__ ptb_all, const int* __restrict__ ptb_off,
                                                  const double* __restrict__ ptab_all,
                                                  const int* __restrict__ ptab_off,
                                                  const uint8_t* __restrict__ kappa_all,
                                                  const double* __restrict__ ctab, const double* __restrict__ axes,
                                                  int nx, int ny, double C_split, double C_merge, double eps_merge,
                                                  int flux_test, uint8_t* __restrict__ kout,
                                                  unsigned long long* __restrict__ hout,
                                                  const int* __restrict__ cell_list) {
    const int nbx = nx / 2, nby = ny / 2, Nb = nbx * nby;
    const bool axes_lds = nx <= CRIT_AXIS && ny <= CRIT_AXIS;
    if (axes_lds) {
        for (int i = threadIdx.x; i < nx; i += blockDim.x) {
            crit_axes[i] = axes[i];
            crit_axes[CRIT_AXIS + i] = axes[nx + i];
        }
        for (int i = threadIdx.x; i < ny; i += blockDim.x) {
            crit_axes[2 * CRIT_AXIS + i] = axes[2 * nx + i];
            crit_axes[3 * CRIT_AXIS + i] = axes[2 * nx + ny + i];
        }
    }
    __syncthreads();
    const int n8x = nbx / 4, n8y = nby / 4, n4x = nbx / 2, n4y = nby / 2;
    for (int ci = item0(); ci < n_cells; ci += istride()) {
        const int c = cell_list ? cell_list[ci] : ci;
        const int lev = cell_lev[c];
        const LevelDesc& L = lvs[lev];
        const size_t row = (size_t)cell_slot[c] * L.stride;
        auto g = rowp<S>(L.g, row);
        auto h = rowp<S>(L.h, row);
        CritCtx cc;
        cc.axes_lds = axes_lds;
        cc.axes = axes;
        cc.ptb = ptb_all + (size_t)ptb_off[lev];
        cc.ptab = ptab_all + (size_t)ptab_off[lev] * NPT;
        cc.klev = kappa_all + (size_t)lev * Nb;
        cc.T1 = ctab;
        cc.T2 = ctab + (size_t)Nb * NCT;
        cc.T3 = cc.T2 + (size_t)n4x * n4y * NCT;
        cc.nx = nx; cc.ny = ny; cc.nbx = nbx; cc.n4x = n4x; cc.n8x = n8x;
        cc.flux_test = flux_test;
        // totals and normalisations over the level's points (Eq. M2; S_r)
        double t[10];
#pragma unroll
        for (int k = 0; k < 10; ++k) t[k] = 0.0;
        for (int p = lane_id(); p < L.N; p += WL) {
            const double* pt = cc.ptab + (size_t)p * NPT;
            const double gv = (double)g[p];
            const double Hv = (double)h[p] + pt[PT_X2] * gv;
            const double w = gp(L.w)[p];
            t[0] += w * gv;
            t[1] += 0.5 * w * Hv;
            const double ag = fabs(gv), aH = 0.5 * fabs(Hv);
            t[2] += ag * pt[PT_AX];
            t[3] += ag * pt[PT_BXX];
            t[4] += ag * pt[PT_BXY];
            t[5] += aH * pt[PT_AX];
            t[6] += ag * pt[PT_AY];
            t[7] += ag * pt[PT_BXY];
            t[8] += ag * pt[PT_BYY];
            t[9] += aH * pt[PT_AY];
        }
        wave_sum<10>(t);
        cc.merge_rho = C_merge * t[0];
        cc.merge_E = C_merge * t[1];
        cc.split_rho = C_split * t[0];
        cc.split_E = C_split * t[1];
        for (int r = 0; r < 4; ++r) cc.epsS[r] = eps_merge * fmax(t[2 + r], t[6 + r]);
        uint8_t* ko = kout + (size_t)c * Nb;
        // Eligible 8x8 blocks, sixteen at a time: four lanes per 8x8 block,
        // one per 4x4 quarter.  A lane keeps the mass and energy sums of its
        // quarter's four 2x2 blocks; the quarter's sums are theirs added in
        // order, the 8x8 block's the four quarters' added in lane order.  The
        // tests then run coarse to fine (Sec. 3.2): the 8x8 block on all four
        // lanes, else each quarter on its lane, else the quarter's 2x2 blocks.
        const int n8 = n8x * n8y;
        for (int t8 = 0; t8 < n8; t8 += WL / 4) {
            const int tb = t8 + (lane_id() >> 2), k = lane_id() & 3;
            const bool act = tb < n8;                     // group-uniform
            const int X8 = act ? tb % n8x : 0, Y8 = act ? tb / n8x : 0;
            const int X4 = 2 * X8 + (k & 1), Y4 = 2 * Y8 + (k >> 1);
            const int c4 = 2 * X4 + nbx * 2 * Y4;         // first 2x2 block of the quarter
            const int k8 = cc.klev[4 * X8 + nbx * 4 * Y8];
            const int k4 = cc.klev[c4];
            const double* T2q = cc.T2 + (size_t)(X4 + n4x * Y4) * NCT;
            const double* T3b = cc.T3 + (size_t)(X8 + n8x * Y8) * NCT;
            // a quarter inside one level point: its sums from its own tables
            double gq = 0.0, Hq = 0.0;
            if (k4 >= 2) crit_gh<S>(cc, g, h, 4 * X4 + nx * 4 * Y4, gq, Hq);
            double c1[4], cH[4], q1, qH;
            if (k4 >= 2) {
                q1 = gq * T2q[CT_W];
                qH = Hq * T2q[CT_W];
#pragma unroll
                for (int j = 0; j < 4; ++j) { c1[j] = 0.0; cH[j] = 0.0; }
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    CritAcc a;
                    acc_zero(a);
                    crit_sum2<S, false>(a, cc, g, h, 2 * X4 + (j & 1), 2 * Y4 + (j >> 1));
                    c1[j] = a.m1;
                    cH[j] = a.mH;
                }
                q1 = (c1[0] + c1[1]) + (c1[2] + c1[3]);
                qH = (cH[0] + cH[1]) + (cH[2] + cH[3]);
            }
            // the 8x8 block's sums: its own tables inside one level point,
            // else the four quarters' sums in lane order
            double e1 = group4_sum(q1), eH = group4_sum(qH);
            if (k8 >= 3) {
                e1 = gq * T3b[CT_W];
                eH = Hq * T3b[CT_W];
            }
            if (!act) continue;
            bool m8 = crit_candidate(cc, e1, eH, 3, 4 * X8 + nbx * 4 * Y8);   // group-uniform
            bool m4 = crit_candidate(cc, q1, qH, 2, c4);                      // the lane's quarter
            // The quarter's half-range fluxes serve both the 8x8 test (summed
            // over the group's four lanes) and the quarter's own test: summed
            // once, when either needs them.
            const bool need8 = m8 && cc.flux_test && k8 < 3;
            CritAcc aq;
            if (need8 || (m4 && cc.flux_test)) {
                acc_zero(aq);
                if (k4 >= 2) acc_table<true>(aq, gq, Hq, T2q);
                else
#pragma unroll 1
                    for (int j = 0; j < 4; ++j) crit_sum2<S, true>(aq, cc, g, h, 2 * X4 + (j & 1), 2 * Y4 + (j >> 1));
            }
            if (m8 && cc.flux_test) {
                CritAcc a;
                if (k8 >= 3) {
                    acc_zero(a);
                    acc_table<true>(a, gq, Hq, T3b);
                } else {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
#pragma unroll
                        for (int d = 0; d < 2; ++d)
#pragma unroll
                            for (int sg = 0; sg < 2; ++sg) a.F[r][d][sg] = group4_sum(aq.F[r][d][sg]);
                }
                a.m1 = e1;
                a.mH = eH;
                m8 = crit_flux_ok(cc, a, T3b);
            }
            uint8_t* q0 = ko + c4;
            if (m8) {
                q0[0] = q0[1] = q0[nbx] = q0[nbx + 1] = 3;
                continue;
            }
            // the lane's 4x4 quarter
            if (m4 && cc.flux_test) {
                aq.m1 = q1;
                aq.mH = qH;
                m4 = crit_flux_ok(cc, aq, T2q);
            }
            if (m4) {
                q0[0] = q0[1] = q0[nbx] = q0[nbx + 1] = 2;
                continue;
            }
            // its 2x2 blocks (inside one level point: their sums from their tables)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int X2 = 2 * X4 + (j & 1), Y2 = 2 * Y4 + (j >> 1);
                const double* T1c = cc.T1 + (size_t)(X2 + nbx * Y2) * NCT;
                if (k4 >= 2) {
                    c1[j] = gq * T1c[CT_W];
                    cH[j] = Hq * T1c[CT_W];
                }
                bool m2 = crit_candidate(cc, c1[j], cH[j], 1, X2 + nbx * Y2);
                if (m2 && cc.flux_test) {
                    CritAcc a;
                    acc_zero(a);
                    if (k4 >= 2) acc_table<true>(a, gq, Hq, T1c);
                    else crit_sum2<S, true>(a, cc, g, h, X2, Y2);
                    a.m1 = c1[j];
                    a.mH = cH[j];
                    m2 = crit_flux_ok(cc, a, T1c);
                }
                ko[X2 + nbx * Y2] = m2 ? (uint8_t)1 : (uint8_t)0;
            }
        }
        // top-level 4x4 blocks outside the 8x8 lattice, then 2x2 blocks outside
        // the 4x4 lattice (odd block counts): one lane per block
        const int n4rest = n4x * n4y - (2 * n8x) * (2 * n8y);
        const int n2rest = nbx * nby - (2 * n4x) * (2 * n4y);
        for (int tb = lane_id(); tb < n4rest + n2rest; tb += WL) {
            int s0, X0 = 0, Y0 = 0;
            if (tb < n4rest) {
                int k = tb, cnt = 0;
                s0 = 2;
                for (int qy = 0; qy < n4y; ++qy)
                    for (int qx = 0; qx < n4x; ++qx) {
                        if (qx < 2 * n8x && qy < 2 * n8y) continue;
                        if (cnt++ == k) { X0 = qx; Y0 = qy; qy = n4y; break; }
                    }
            } else {
                int k = tb - n4rest, cnt = 0;
                s0 = 1;
                for (int yy = 0; yy < nby; ++yy)
                    for (int xx = 0; xx < nbx; ++xx) {
                        if (xx < 2 * n4x && yy < 2 * n4y) continue;
                        if (cnt++ == k) { X0 = xx; Y0 = yy; yy = nby; break; }
                    }
            }
            if (s0 == 2) {
                uint8_t* q0 = ko + 2 * X0 + nbx * 2 * Y0;
                if (crit_test<S>(cc, g, h, 2, X0, Y0)) {
                    q0[0] = q0[1] = q0[nbx] = q0[nbx + 1] = 2;
                } else {
                    for (int j = 0; j < 4; ++j) {
                        const int X2 = 2 * X0 + (j & 1), Y2 = 2 * Y0 + (j >> 1);
                        ko[X2 + nbx * Y2] = crit_test<S>(cc, g, h, 1, X2, Y2) ? (uint8_t)1 : (uint8_t)0;
                    }
                }
            } else {
                ko[X0 + nbx * Y0] = crit_test<S>(cc, g, h, 1, X0, Y0) ? (uint8_t)1 : (uint8_t)0;
            }
        }
        __threadfence_block();
        unsigned long long hs = 0ull;
        for (int b = lane_id(); b < Nb; b += WL) hs += mix64(((unsigned long long)b << 2) | ko[b]);
        for (int off = 32; off > 0; off >>= 1) hs += __shfl_xor(hs, off, WL);
        if (lane_id() == 0) hout[c] = hs;
    }
}

__global__ void k_gather_rows_u8(const uint8_t* __restrict__ src, int width, const int* __restrict__ rows, int n,
                                 uint8_t* __restrict__ dst) {
    for (int r = item0(); r < n; r += istride())
        for (int k = lane_id(); k < width; k += WL) dst[(size_t)r * width + k] = src[(size_t)rows[r] * width + k];
}

// Row gather in 16-byte units: dst row r is src row rows[r].
__global__ void k_gather_rows_16(const uint4* __restrict__ src, int width16, const int* __restrict__ rows, int n,
                                 uint4* __restrict__ dst) {
    for (int r = item0(); r < n; r += istride()) {
        const uint4* a = src + (size_t)rows[r] * width16;
        uint4* b = dst + (size_t)r * width16;
        for (int k = lane_id(); k < width16; k += WL) b[k] = a[k];
    }
}

__global__ void k_compare_rows_u8(const uint8_t* __restrict__ all, int width, const int* __restrict__ rep_of_cell,
                                  const uint8_t* __restrict__ reps, int n, unsigned long long* mismatch) {
    for (int c = item0(); c < n; c += istride()) {
        int bad = 0;
        const uint8_t* a = all + (size_t)c * width;
        const uint8_t* r = reps + (size_t)rep_of_cell[c] * width;
        for (int k = lane_id(); k < width; k += WL) bad |= (a[k] != r[k]);
        if (__any(bad) && lane_id() == 0) atomicAdd(mismatch, 1ull);
    }
}

// ---------------------------------------------------------------------------
// the persistent step: one launch per step
// ---------------------------------------------------------------------------
// Grid-wide barrier.  Every workgroup of the launch is resident (the grid is
// sized from this kernel's occupancy), so all of them arrive.  The agent-scope
// fences write the arriving workgroup's results back past its XCD's L2 and
// make the others' visible after the wait.  The wait is bounded: past the
// bound the sticky error flag sync[1] is set and the barrier is left, the step
// is then invalid and the host reports it; no wave waits for ever.
__device__ __forceinline__ void grid_barrier(unsigned int* sync, unsigned int& phase) {
    __syncthreads();
    ++phase;
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned int target = phase * gridDim.x;
        atomicAdd(sync, 1u);
        unsigned int k = 0;
        while (__hip_atomic_load(sync, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(32);
            if (++k > (1u << 21)) {
                atomicOr(sync + 1, 1u);
                break;
            }
        }
        __threadfence();
    }
    __syncthreads();
}

// The fused step of one time step (neighbour rows; cross-level and
// same-level faces; update with the next step's cell stage) as one launch
// over the work lists of StepArgs, whose pointers and counts are read from
// device memory: a captured launch stays valid when an adaptation replaces
// the level set.  Stages are separated by grid barriers.  The cross-level
// faces (few, long) take the first slots of the face stage's index space.
// Same arithmetic as the four fused-step kernels.
template <typename S, int U, int MINW, int CM, int MK>
__global__ __launch_bounds__(BS, MINW) void k_step_persistent(const StepArgs* __restrict__ A, Phys ph) {
    const int first = item0(), stride = istride();
    unsigned int phase = 0;
    ghost_items<S>(A->lvs, A->ghosts, A->n_ghosts, A->cell_lev, A->cell_slot, A->params, ph, A->neg, first, stride);
    grid_barrier(A->sync, phase);
    const int nx = A->n_xfaces;
    xface_items<S, U, MK>(A->lvs, A->xfaces, nx, A->cell_slot, A->cell_nbr, A->geom, A->params, ph, A->neg, first,
                          stride);
    const int fstart = ((first - nx) % stride + stride) % stride;
    face_full_items<S, U, CM, MK>(A->lvs, A->faces, A->n_faces, A->cell_slot, A->cell_nbr, A->geom, A->params,
                                  A->bcs, ph, A->fpar, fstart, stride);
    grid_barrier(A->sync, phase);
    update_cell_items<S, U, CM>(A->lvs, A->cell_lev, A->cell_slot, A->order, A->n_cells, A->geom, A->cell_frow,
                                A->faces, A->fpar, A->params, ph, A->cmom, first, stride);
}

// Arrivals of the barrier counter back to zero before a launch (a kernel, so
// the captured step holds no memset node).
__global__ void k_sync_reset(unsigned int* sync) {
    if (threadIdx.x == 0) sync[0] = 0u;
}

template <typename KF>
static hipError_t persistent_grid(KF kernel, int* grid) {
    int dev = 0, ncu = 0, nb = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, BS, 0);
    if (e != hipSuccess) return e;
    const int g = ncu * nb / NXCD * NXCD;
    if (g < NXCD) return hipErrorInvalidConfiguration;
    *grid = g;
    return hipSuccess;
}

#define MLVS_PERSISTENT(S_, U_, C_, MK_)                                                         \
    do {                                                                                        \
        auto kf = k_step_persistent<S_, U_, 2, C_, MK_>;                                         \
        if ((e = persistent_grid(kf, &g)) != hipSuccess) return e;                               \
        hipLaunchKernelGGL(kf, dim3(g), dim3(BS), 0, st, A, ph);                                 \
    } while (0)
#define MLVS_PERSISTENT_C(S_, U_, MK_)                                                           \
    do {                                                                                        \
        if (ph.compat == 8) MLVS_PERSISTENT(S_, U_, 8, MK_);                                     \
        else MLVS_PERSISTENT(S_, U_, 4, MK_);                                                    \
    } while (0)
#define MLVS_PERSISTENT_U(S_)                                                                    \
    do {                                                                                        \
        if (ph.mesh_kind) MLVS_PERSISTENT_C(S_, 1, 1);                                           \
        else if (var == 1) MLVS_PERSISTENT_C(S_, 2, 0);                                          \
        else MLVS_PERSISTENT_C(S_, 1, 0);                                                        \
    } while (0)

int persistent_variant_count() { return 2; }

hipError_t launch_step_persistent(int prec, hipStream_t st, const StepArgs* A, unsigned int* sync, Phys ph, int var,
                                  int* grid_used) {
    hipError_t e = hipSuccess;
    int g = 0;
    hipLaunchKernelGGL(k_sync_reset, dim3(1), dim3(64), 0, st, sync);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (prec == 32) MLVS_PERSISTENT_U(float);
    else MLVS_PERSISTENT_U(double);
    if (grid_used) *grid_used = g;
    return hipGetLastError();
}

hipError_t launch_xface(int prec, hipStream_t st, const LevelDesc* lv, const XFaceItem* items, int n,
                        const int* cell_slot, const int* cell_nbr, const CellGeom* geom, const double* params,
                        Phys ph, unsigned long long* neg, int var) {
    if (n <= 0) return hipSuccess;
    MLVS_DISPATCH_VM(prec, var, ph.mesh_kind, k_xface, dim3(grid_for(n)), dim3(BS), 0, st, lv, items, n, cell_slot,
                     cell_nbr, geom, params, ph, neg);
    return hipGetLastError();
}

hipError_t launch_criterion(int prec, hipStream_t st, const LevelDesc* lv, const int* cell_lev, const int* cell_slot,
                            int n_cells, const int* pt_of_base_all, const int* pt_off, const double* ptab_all,
                            const int* ptab_off, const uint8_t* kappa_all, const double* ctab, const double* axes,
                            int nx, int ny, double C_split, double C_merge, double eps_merge, int flux_test,
                            uint8_t* kappa_out, unsigned long long* hash_out, const int* cell_list) {
    if (n_cells <= 0) return hipSuccess;
    MLVS_DISPATCH(prec, k_criterion, dim3(grid_for(n_cells)), dim3(BS), 0, st, lv, cell_lev, cell_slot, n_cells,
                  pt_of_base_all, pt_off, ptab_all, ptab_off, kappa_all, ctab, axes, nx, ny, C_split, C_merge,
                  eps_merge, flux_test, kappa_out, hash_out, cell_list);
    return hipGetLastError();
}

hipError_t launch_gather_rows_16(hipStream_t st, const void* src, int width16, const int* rows, int n, void* dst) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_rows_16, dim3(grid_for(n)), dim3(BS), 0, st, static_cast<const uint4*>(src), width16,
                       rows, n, static_cast<uint4*>(dst));
    return hipGetLastError();
}

hipError_t launch_gather_rows_u8(hipStream_t st, const uint8_t* src, int width, const int* rows, int n,
                                 uint8_t* dst) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_rows_u8, dim3(grid_for(n)), dim3(BS), 0, st, src, width, rows, n, dst);
    return hipGetLastError();
}

hipError_t launch_compare_rows_u8(hipStream_t st, const uint8_t* all, int width, const int* rep_of_cell,
                                  const uint8_t* reps, int n, unsigned long long* mismatch) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_compare_rows_u8, dim3(grid_for(n)), dim3(BS), 0, st, all, width, rep_of_cell, reps, n,
                       mismatch);
    return hipGetLastError();
}

}  // namespace mlvs
