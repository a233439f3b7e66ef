// Host side of libmlvs: the C ABI, mesh geometry, velocity levels, projection
// tables, clustering and the per-step launch sequence.  All per-velocity work
// runs in the kernels of kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <thread>
#include <unistd.h>
#include <mutex>
#include <condition_variable>
#include <functional>
#include <unordered_map>
#include <vector>

#include "../../include/mlvs.h"
#include "mlvs_impl.h"

using namespace mlvs;

namespace {

thread_local std::string g_last_error;

// MLVS_TIMING=1 in the environment: host wall-clock marks of the adaptation's
// parts on stderr (diagnostics only).
struct Marks {
    bool on = std::getenv("MLVS_TIMING") != nullptr;
    std::chrono::steady_clock::time_point t = std::chrono::steady_clock::now();
    void mark(const char* what, hipStream_t st) {
        if (!on) return;
        (void)hipStreamSynchronize(st);
        const auto now = std::chrono::steady_clock::now();
        std::fprintf(stderr, "[mlvs] %-28s %9.3f ms\n", what, std::chrono::duration<double, std::milli>(now - t).count());
        t = now;
    }
};

struct Fail {
    int code;
    std::string msg;
};

[[noreturn]] void fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    throw Fail{code, buf};
}

void hip_check(hipError_t e, const char* what) {
    if (e != hipSuccess) fail(MLVS_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

template <typename F>
mlvs_status guarded(F&& f) {
    try {
        f();
        return MLVS_OK;
    } catch (const Fail& e) {
        g_last_error = e.msg;
        return e.code;
    } catch (const std::bad_alloc&) {
        g_last_error = "host allocation failed";
        return MLVS_E_OOM;
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return MLVS_E_STATE;
    }
}

// ---------------------------------------------------------------------------
// quadrature (Sec. 2.3)
// ---------------------------------------------------------------------------
void newton_cotes(int n, double a, double* x, double* w) {
    if (n < 2) fail(MLVS_E_ARG, "need at least two velocity nodes");
    if (n % 2 == 0) {
        const double hh = 2.0 * a / n;
        for (int k = 0; k < n; ++k) { x[k] = -a + hh * (k + 0.5); w[k] = hh; }
        return;
    }
    const double hh = 2.0 * a / (n - 1);
    for (int k = 0; k < n; ++k) { x[k] = a * (2.0 * k - (n - 1)) / (n - 1); w[k] = 0.0; }
    if ((n - 1) % 4 == 0) {
        const double c[5] = {7, 32, 12, 32, 7};
        for (int p = 0; p < n - 1; p += 4)
            for (int k = 0; k < 5; ++k) w[p + k] += c[k] * (2.0 * hh / 45.0);
    } else {
        const double c[3] = {1, 4, 1};
        for (int p = 0; p < n - 1; p += 2)
            for (int k = 0; k < 3; ++k) w[p + k] += c[k] * (hh / 3.0);
    }
}

// Gauss-Hermite nodes/weights for weight exp(-x^2) by Newton on the
// orthonormal Hermite recurrence; scaled to integrate f itself.
void gauss_hermite(int n, double R, double T0, double* x, double* w) {
    if (n < 1 || n > 400) fail(MLVS_E_ARG, "Gauss-Hermite order out of range");
    std::vector<double> xs(n), ws(n);
    const double pim4 = 0.7511255444649425;   // pi^(-1/4)
    double z = 0.0;
    for (int i = 0; i < (n + 1) / 2; ++i) {
        if (i == 0) z = std::sqrt(2.0 * n + 1.0) - 1.85575 * std::pow(2.0 * n + 1.0, -0.16667);
        else if (i == 1) z -= 1.14 * std::pow((double)n, 0.426) / z;
        else if (i == 2) z = 1.86 * z - 0.86 * xs[0];
        else if (i == 3) z = 1.91 * z - 0.91 * xs[1];
        else z = 2.0 * z - xs[i - 2];
        double pp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p1 = pim4, p2 = 0.0;
            for (int j = 0; j < n; ++j) {
                const double p3 = p2;
                p2 = p1;
                p1 = z * std::sqrt(2.0 / (j + 1)) * p2 - std::sqrt((double)j / (j + 1)) * p3;
            }
            pp = std::sqrt(2.0 * n) * p2;
            const double z1 = z;
            z = z1 - p1 / pp;
            if (std::fabs(z - z1) <= 1e-15 * std::max(1.0, std::fabs(z))) break;
        }
        xs[i] = z;
        xs[n - 1 - i] = -z;
        ws[i] = 2.0 / (pp * pp);
        ws[n - 1 - i] = ws[i];
    }
    const double c = std::sqrt(2.0 * R * T0);
    for (int i = 0; i < n; ++i) {
        const double xi = xs[n - 1 - i];   // ascending
        x[i] = c * xi;
        w[i] = c * ws[n - 1 - i] * std::exp(xi * xi);
    }
}

// ---------------------------------------------------------------------------
// small dense helpers
// ---------------------------------------------------------------------------
// Inverse of a row-major n x n matrix (n <= 8) by Gauss-Jordan elimination with
// partial pivoting; false if singular.
bool invert_n(const double* A, int n, double* inv) {
    double M[8][16];
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < 2 * n; ++c) M[r][c] = c < n ? A[r * n + c] : (c - n == r ? 1.0 : 0.0);
    for (int k = 0; k < n; ++k) {
        int p = k;
        for (int i = k + 1; i < n; ++i)
            if (std::fabs(M[i][k]) > std::fabs(M[p][k])) p = i;
        if (M[p][k] == 0.0) return false;
        if (p != k)
            for (int c = 0; c < 2 * n; ++c) std::swap(M[k][c], M[p][c]);
        const double d = M[k][k];
        for (int c = 0; c < 2 * n; ++c) M[k][c] /= d;
        for (int i = 0; i < n; ++i) {
            if (i == k) continue;
            const double f = M[i][k];
            for (int c = 0; c < 2 * n; ++c) M[i][c] -= f * M[k][c];
        }
    }
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) inv[r * n + c] = M[r][c + n];
    return true;
}

bool invert4(const double* A, double* inv) { return invert_n(A, 4, inv); }

// ---------------------------------------------------------------------------
// device memory
// ---------------------------------------------------------------------------
struct DevMem {
    mlvs_device dev{};
    size_t bytes = 0;
    std::unordered_map<void*, size_t> live;

    void* alloc(size_t n) {
        if (n == 0) n = 8;
        n = (n + 255) & ~size_t(255);
        void* p = nullptr;
        if (dev.alloc) {
            p = dev.alloc(n, dev.user);
            if (!p) fail(MLVS_E_OOM, "device allocation of %zu bytes failed", n);
        } else {
            if (hipMalloc(&p, n) != hipSuccess) fail(MLVS_E_OOM, "hipMalloc of %zu bytes failed", n);
        }
        live[p] = n;
        bytes += n;
        return p;
    }
    void release(void* p) {
        if (!p) return;
        auto it = live.find(p);
        if (it == live.end()) return;
        bytes -= it->second;
        live.erase(it);
        if (dev.free) dev.free(p, dev.user);
        else (void)hipFree(p);
    }
    void release_all() {
        std::vector<void*> ps;
        for (auto& kv : live) ps.push_back(kv.first);
        for (void* p : ps) release(p);
    }
};

template <typename T>
T* upload(DevMem& dm, const std::vector<T>& v, hipStream_t st) {
    T* d = static_cast<T*>(dm.alloc(sizeof(T) * std::max<size_t>(v.size(), 1)));
    if (!v.empty()) hip_check(hipMemcpyAsync(d, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, st), "upload");
    return d;
}

// ---------------------------------------------------------------------------
// velocity levels (Sec. 3.2)
// ---------------------------------------------------------------------------
struct Base {
    int nx = 0, ny = 0, N = 0, nbx = 0, nby = 0, Nb = 0;
    std::vector<double> x, y, w;     // per base point
    std::vector<double> axes;        // the tensor grid's axes: x [nx], wx [nx], y [ny], wy [ny]
    std::vector<double> ctab;        // criterion: per aligned block of scales 1, 2, 3 (see block_tables)
};

// Criterion tables of the aligned blocks of V_base (scale 1: N_b 2x2 blocks,
// then the eligible 4x4 and 8x8 blocks), 15 values each: sum w, the velocity
// centroid (sum w xi_x, sum w xi_y) / sum w, then for d = x, y and the
// half-ranges s = (xi_d >= 0, xi_d <= 0) P[d][s] = sum w xi_d, then
// Q[d][s][e] = sum w xi_d xi_e.
void block_tables(Base& B) {
    B.ctab.clear();
    const int n4x = B.nbx / 2, n4y = B.nby / 2, n8x = B.nbx / 4, n8y = B.nby / 4;
    auto put = [&](int s, int X, int Y) {
        double t[15] = {0};
        const int size = 1 << s;
        for (int iy = Y * size; iy < Y * size + size; ++iy)
            for (int ix = X * size; ix < X * size + size; ++ix) {
                const int b = ix + B.nx * iy;
                const double w = B.w[b], xd[2] = {B.x[b], B.y[b]};
                t[0] += w;
                t[1] += w * xd[0];
                t[2] += w * xd[1];
                for (int d = 0; d < 2; ++d)
                    for (int sg = 0; sg < 2; ++sg) {
                        if (!(sg == 0 ? xd[d] >= 0 : -xd[d] >= 0)) continue;
                        t[3 + 2 * d + sg] += w * xd[d];
                        t[7 + 4 * d + 2 * sg] += w * xd[d] * xd[0];
                        t[7 + 4 * d + 2 * sg + 1] += w * xd[d] * xd[1];
                    }
            }
        t[1] /= t[0];
        t[2] /= t[0];
        B.ctab.insert(B.ctab.end(), t, t + 15);
    };
    for (int Y = 0; Y < B.nby; ++Y)
        for (int X = 0; X < B.nbx; ++X) put(1, X, Y);
    for (int Y = 0; Y < n4y; ++Y)
        for (int X = 0; X < n4x; ++X) put(2, X, Y);
    for (int Y = 0; Y < n8y; ++Y)
        for (int X = 0; X < n8x; ++X) put(3, X, Y);
    if (B.ctab.empty()) B.ctab.assign(15, 0.0);
}

struct Level {
    std::vector<uint8_t> kappa;
    int N = 0;
    std::vector<double> xi_x, xi_y, w;
    std::vector<int> pt_of_base;
    std::vector<int> mem_off, mem_idx;     // base members per point (ascending)
    std::vector<int> canon_of;             // device point -> canonical point (I/O order)
    std::vector<double> crit_tab;          // per point: |xi_p|^2, sum w|x|, w|y|, w x^2, w|xy|, w y^2 over members
    double Minv[16];
    double G6inv[36], B36[18], H3inv[9];   // nine-moment mapping (see build_level)
    bool is_iface = false;
    bool geo_in_arena = false;             // device geometry lives in a build's staging block
    // device
    double *d_x = nullptr, *d_y = nullptr, *d_w = nullptr;
    float* d_xy = nullptr;                 // (xi_x, xi_y) pairs in float, for FP32 storage
    int* d_pt_of_base = nullptr;
    int stride = 0;
    int n_cells = 0, n_rows = 0, n_ghost = 0;
    void *g = nullptr, *h = nullptr, *fg = nullptr, *fh = nullptr;
    void *Fg = nullptr, *Fh = nullptr;
    size_t rows_alloc = 0, ghost_alloc = 0;
};

void check_kappa(const Base& B, const uint8_t* k) {
    for (int b = 0; b < B.Nb; ++b)
        if (k[b] > 3) fail(MLVS_E_ARG, "kappa value out of range");
    const int n8x = B.nbx / 4, n8y = B.nby / 4, n4x = B.nbx / 2, n4y = B.nby / 2;
    for (int by = 0; by < B.nby; ++by)
        for (int bx = 0; bx < B.nbx; ++bx) {
            const int v = k[bx + B.nbx * by];
            if (v == 3 && !(bx < 4 * n8x && by < 4 * n8y)) fail(MLVS_E_ARG, "8x8 merge outside an eligible block");
            if (v == 2 && !(bx < 2 * n4x && by < 2 * n4y)) fail(MLVS_E_ARG, "4x4 merge outside an eligible block");
        }
    for (int oy = 0; oy < n8y; ++oy)
        for (int ox = 0; ox < n8x; ++ox) {
            int c3 = 0;
            for (int j = 0; j < 4; ++j)
                for (int i = 0; i < 4; ++i) c3 += k[4 * ox + i + B.nbx * (4 * oy + j)] == 3;
            if (c3 != 0 && c3 != 16) fail(MLVS_E_ARG, "inconsistent 8x8 block in kappa");
        }
    for (int qy = 0; qy < n4y; ++qy)
        for (int qx = 0; qx < n4x; ++qx) {
            int c2 = 0, cge = 0;
            for (int j = 0; j < 2; ++j)
                for (int i = 0; i < 2; ++i) {
                    const int v = k[2 * qx + i + B.nbx * (2 * qy + j)];
                    c2 += v == 2;
                    cge += v >= 2;
                }
            if (c2 != 0 && cge != 4) fail(MLVS_E_ARG, "inconsistent 4x4 block in kappa");
        }
}

// Velocity and weight of the point made of the 2^s x 2^s block of base points
// whose first (smallest) index is b0, or of the single point b0 when s = 0:
// the w-weighted mean and the sum, members taken in ascending index order.  A
// component of a merged point that cancels by the grid's symmetry (within
// 1e-12 of the members' largest |coordinate|) is exactly zero rather than the
// rounding residue of the mean, so that xi . n = 0 on faces along the axes is
// decided as in exact arithmetic.
void merged_point(const Base& B, int b0, int s, double& ws, double& x, double& y) {
    const int size = 1 << s;
    double sx = 0.0, sy = 0.0, ex = 0.0, ey = 0.0;
    ws = 0.0;
    for (int iy = 0; iy < size; ++iy)
        for (int ix = 0; ix < size; ++ix) ws += B.w[b0 + ix + B.nx * iy];
    for (int iy = 0; iy < size; ++iy)
        for (int ix = 0; ix < size; ++ix) {
            const int b = b0 + ix + B.nx * iy;
            sx += B.w[b] * B.x[b];
            sy += B.w[b] * B.y[b];
            ex = std::max(ex, std::fabs(B.x[b]));
            ey = std::max(ey, std::fabs(B.y[b]));
        }
    x = sx / ws + 0.0;                  // + 0.0: no negative zeros
    y = sy / ws + 0.0;
    if (s > 0) {
        if (std::fabs(x) <= 1e-12 * ex) x = 0.0;
        if (std::fabs(y) <= 1e-12 * ey) y = 0.0;
    }
}

std::unique_ptr<Level> build_level(const Base& B, const std::vector<uint8_t>& kappa) {
    auto L = std::make_unique<Level>();
    L->kappa = kappa;
    // a level point is an aligned 2^s block (s = 1, 2, 3) or a single base
    // point (s = 0), named by its first base index
    struct Grp { int b0, s; };
    // scale of the point starting at each base index (-1: inside another point)
    std::vector<signed char> start(B.N, 0);
    auto block = [&](int s, int bx, int by) {
        const int size = 1 << s, b0 = bx * size + B.nx * by * size;
        for (int iy = 0; iy < size; ++iy)
            for (int ix = 0; ix < size; ++ix) start[b0 + ix + B.nx * iy] = -1;
        start[b0] = (signed char)s;
    };
    auto kap = [&](int bx, int by) { return (int)kappa[bx + B.nbx * by]; };
    if (B.Nb > 0) {
        for (int oy = 0; oy < B.nby / 4; ++oy)
            for (int ox = 0; ox < B.nbx / 4; ++ox)
                if (kap(4 * ox, 4 * oy) == 3) block(3, ox, oy);
        for (int qy = 0; qy < B.nby / 2; ++qy)
            for (int qx = 0; qx < B.nbx / 2; ++qx)
                if (kap(2 * qx, 2 * qy) == 2) block(2, qx, qy);
        for (int by = 0; by < B.nby; ++by)
            for (int bx = 0; bx < B.nbx; ++bx)
                if (kap(bx, by) == 1) block(1, bx, by);
    }
    // canonical order (the interface order of every per-point array): ascending
    // smallest base index of each point
    std::vector<Grp> groups;
    groups.reserve(B.N);
    for (int b = 0; b < B.N; ++b)
        if (start[b] >= 0) groups.push_back({b, start[b]});
    const int n = (int)groups.size();
    std::vector<double> pw(n), px(n), py(n);
    for (int p = 0; p < n; ++p) merged_point(B, groups[p].b0, groups[p].s, pw[p], px[p], py[p]);
    // device order: by polar angle of the point's velocity, then speed, then
    // canonical index.  For any face normal n the points with xi . n > 0 then
    // form one arc of consecutive indices (two pieces if it wraps), so almost
    // every 64-point chunk of a face has a single upwind side.
    std::vector<int> ord(n);
    {
        struct Key { double ang, r2; int p; };
        std::vector<Key> key(n);
        for (int p = 0; p < n; ++p) key[p] = {std::atan2(py[p], px[p]), px[p] * px[p] + py[p] * py[p], p};
        std::sort(key.begin(), key.end(), [](const Key& a, const Key& b) {
            if (a.ang != b.ang) return a.ang < b.ang;
            if (a.r2 != b.r2) return a.r2 < b.r2;
            return a.p < b.p;
        });
        for (int d = 0; d < n; ++d) ord[d] = key[d].p;
    }
    L->N = n;
    L->canon_of = ord;
    L->pt_of_base.assign(B.N, -1);
    L->mem_off.assign(n + 1, 0);
    L->mem_idx.reserve(B.N);
    L->xi_x.resize(n);
    L->xi_y.resize(n);
    L->w.resize(n);
    for (int d = 0; d < n; ++d) {
        const Grp& G = groups[ord[d]];
        const int size = 1 << G.s;
        for (int iy = 0; iy < size; ++iy)
            for (int ix = 0; ix < size; ++ix) {
                const int b = G.b0 + ix + B.nx * iy;
                L->pt_of_base[b] = d;
                L->mem_idx.push_back(b);
            }
        L->w[d] = pw[ord[d]];
        L->xi_x[d] = px[ord[d]];
        L->xi_y[d] = py[ord[d]];
        L->mem_off[d + 1] = (int)L->mem_idx.size();
    }
    // criterion tables of the points (normalisations S_r of Eq. merge-transport-error)
    L->crit_tab.assign(6 * (size_t)L->N, 0.0);
    for (int p = 0; p < L->N; ++p) {
        double* t = &L->crit_tab[6 * (size_t)p];
        t[0] = L->xi_x[p] * L->xi_x[p] + L->xi_y[p] * L->xi_y[p];
        for (int k = L->mem_off[p]; k < L->mem_off[p + 1]; ++k) {
            const int b = L->mem_idx[k];
            const double w = B.w[b], ax = std::fabs(B.x[b]), ay = std::fabs(B.y[b]);
            t[1] += w * ax;
            t[2] += w * ay;
            t[3] += w * ax * ax;
            t[4] += w * ax * ay;
            t[5] += w * ay * ay;
        }
    }
    // state-independent four-moment mapping matrix (Eqs. raw_four_g_basis, raw_four_gh_coupling)
    double A[16] = {0};
    for (int p = 0; p < L->N; ++p) {
        const double x = L->xi_x[p], y = L->xi_y[p], w = L->w[p], x2 = x * x + y * y;
        const double psi[4] = {1.0, x, y, 0.5 * x2}, phi[4] = {1.0, x, y, x2};
        for (int r = 0; r < 4; ++r)
            for (int c = 0; c < 4; ++c) A[r * 4 + c] += w * psi[r] * phi[c];
    }
    if (!invert4(A, L->Minv)) std::fill(L->Minv, L->Minv + 16, 0.0);
    // state-independent matrices of the nine-moment mapping (Eqs. raw_six_g_basis,
    // raw_three_h_basis, mapping_h_residual_correction): g basis [1, x, y, x^2,
    // y^2, xy] against the same six g moments; h basis [1, x, y] against the
    // energy and energy-flux moments (1/2 weight); B couples the g correction
    // into those three through 1/2 |xi|^2 dg.
    double Ag[36] = {0}, Ah[9] = {0};
    std::fill(L->B36, L->B36 + 18, 0.0);
    for (int p = 0; p < L->N; ++p) {
        const double x = L->xi_x[p], y = L->xi_y[p], w = L->w[p], x2 = x * x + y * y;
        const double pg[6] = {1.0, x, y, x * x, y * y, x * y}, ph3[3] = {1.0, x, y};
        for (int r = 0; r < 6; ++r)
            for (int c = 0; c < 6; ++c) Ag[r * 6 + c] += w * pg[r] * pg[c];
        for (int r = 0; r < 3; ++r) {
            for (int c = 0; c < 3; ++c) Ah[r * 3 + c] += 0.5 * w * ph3[r] * ph3[c];
            for (int c = 0; c < 6; ++c) L->B36[r * 6 + c] += w * x2 * ph3[r] * pg[c];
        }
    }
    if (!invert_n(Ag, 6, L->G6inv)) std::fill(L->G6inv, L->G6inv + 36, 0.0);
    if (!invert_n(Ah, 3, L->H3inv)) std::fill(L->H3inv, L->H3inv + 9, 0.0);
    return L;
}

// dst <- src projection table (CSR over dst points).
struct HostTable {
    std::vector<int> off, idx;
    std::vector<double> frac;
};

// build_level through the context's cache (a level is a function of the base
// grid and its mask alone).  The returned level is a fresh copy with no
// device memory.
std::unique_ptr<Level> level_of_mask(mlvs_ctx c, const std::vector<uint8_t>& kappa);

HostTable make_table(const Level& dst, const Level& src) {
    HostTable t;
    t.off.reserve(dst.N + 1);
    t.idx.reserve(dst.N);
    t.frac.reserve(dst.N);
    t.off.push_back(0);
    // stamp[a] = the last dst point that listed source point a (O(members) per point)
    std::vector<int> stamp(src.N, -1);
    for (int P = 0; P < dst.N; ++P) {
        const int b0 = dst.mem_idx[dst.mem_off[P]];
        const int a0 = src.pt_of_base[b0];
        bool single = true;
        for (int e = dst.mem_off[P]; e < dst.mem_off[P + 1]; ++e)
            if (src.pt_of_base[dst.mem_idx[e]] != a0) { single = false; break; }
        if (single) {
            t.idx.push_back(a0);
            t.frac.push_back(1.0);
        } else {
            for (int e = dst.mem_off[P]; e < dst.mem_off[P + 1]; ++e) {
                const int a = src.pt_of_base[dst.mem_idx[e]];
                if (stamp[a] == P) continue;
                stamp[a] = P;
                t.idx.push_back(a);
                t.frac.push_back(src.w[a] / dst.w[P]);
            }
        }
        t.off.push_back((int)t.idx.size());
    }
    return t;
}

struct DevTable {
    int* off = nullptr;
    int* idx = nullptr;
    double* frac = nullptr;
    PairTable view() const { return PairTable{off, idx, frac}; }
};

// Host worker threads for the adaptation's parallel passes, started on first
// use and kept (starting a thread costs tens of microseconds, and an
// adaptation runs several passes).  run(nt, f) calls f(t) for t in [0, nt),
// t = 0 on the calling thread, and returns when every call has returned;
// calls of run are serialised.
class HostPool {
public:
    static HostPool& get() {
        static HostPool pool;
        return pool;
    }
    int size() const { return (int)workers_.size() + 1; }
    void run(int nt, const std::function<void(int)>& f) {
        std::lock_guard<std::mutex> serial(run_m_);
        if (getpid() != pid_) {                    // a forked child has no workers
            for (int t = 0; t < nt; ++t) f(t);
            return;
        }
        nt = std::min(nt, size());
        if (nt <= 1) { f(0); return; }
        {
            std::lock_guard<std::mutex> g(m_);
            job_ = &f;
            active_ = nt - 1;
            pending_ = nt - 1;
            ++gen_;
        }
        cv_.notify_all();
        f(0);
        std::unique_lock<std::mutex> lk(m_);
        done_.wait(lk, [&] { return pending_ == 0; });
        job_ = nullptr;
    }
    ~HostPool() {
        {
            std::lock_guard<std::mutex> g(m_);
            stop_ = true;
            ++gen_;
        }
        cv_.notify_all();
        for (auto& t : workers_) t.join();
    }

private:
    HostPool() : pid_(getpid()) {
        const unsigned hw = std::max(1u, std::min(8u, std::thread::hardware_concurrency()));
        for (unsigned i = 1; i < hw; ++i) workers_.emplace_back([this, i] { loop((int)i); });
    }
    void loop(int idx) {
        unsigned long long seen = 0;
        for (;;) {
            const std::function<void(int)>* f = nullptr;
            {
                std::unique_lock<std::mutex> lk(m_);
                cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
                if (stop_) return;
                seen = gen_;
                if (idx > active_) continue;           // not needed in this run
                f = job_;
            }
            (*f)(idx);
            std::lock_guard<std::mutex> g(m_);
            if (--pending_ == 0) done_.notify_one();
        }
    }
    std::vector<std::thread> workers_;
    std::mutex m_, run_m_;
    std::condition_variable cv_, done_;
    const std::function<void(int)>* job_ = nullptr;
    int active_ = 0, pending_ = 0;
    unsigned long long gen_ = 0;
    bool stop_ = false;
    pid_t pid_;
};

// Run f(lo, hi) over [0, n) split into contiguous ranges on the host pool,
// each range at least `grain` long (one range on the calling thread when n is
// small).  f must only write its own range.
template <class F>
void parallel_ranges(int n, int grain, F&& f) {
    HostPool& P = HostPool::get();
    const int nt = (int)std::min<long>(P.size(), std::max(1, n / std::max(grain, 1)));
    if (nt <= 1) { f(0, n); return; }
    const std::function<void(int)> job = [&](int t) {
        f((int)((long)n * t / nt), (int)((long)n * (t + 1) / nt));
    };
    P.run(nt, job);
}

// Host image of the many small arrays a level set needs on the device (work
// lists, projection tables, descriptors): one device block and one copy per
// build instead of one allocation and copy per array.  Pieces are 256-byte
// aligned; the block starts with a 256-byte pad so no piece shares the block's
// address.
// Staging area of one upload: a host image of a device block, written in
// place, then copied with one hipMemcpyAsync.  It lives in pinned memory kept
// by the context between builds (a fresh pageable image cost page faults and
// reallocation copies on every adaptation, and its copy ran at pageable
// speed); it grows geometrically and only ever grows.
struct Stage {
    uint8_t* p = nullptr;
    size_t cap = 0, size = 256;
    Stage(uint8_t*& buf, size_t& capacity) : p(buf), cap(capacity), bref(buf), cref(capacity) {}
    ~Stage() { bref = p; cref = cap; }
    Stage(const Stage&) = delete;
    Stage& operator=(const Stage&) = delete;
    void reserve(size_t n) {
        if (n <= cap) return;
        const size_t want = std::max(n, std::max(2 * cap, (size_t)16 << 20));
        uint8_t* q = nullptr;
        hip_check(hipHostMalloc((void**)&q, want, hipHostMallocDefault), "pinned alloc");
        if (p) {
            std::memcpy(q, p, size);
            (void)hipHostFree(p);
        }
        p = q;
        cap = want;
    }
    size_t put(const void* src, size_t n) {
        const size_t off = (size + 255) & ~size_t(255);
        reserve(off + std::max<size_t>(n, 1));
        if (src && n) std::memcpy(p + off, src, n);
        size = off + std::max<size_t>(n, 1);
        return off;
    }
    template <typename T>
    size_t put(const std::vector<T>& v) { return put(v.data(), sizeof(T) * v.size()); }
    template <typename T>
    void fill(size_t off, const std::vector<T>& v) {
        if (!v.empty()) std::memcpy(p + off, v.data(), sizeof(T) * v.size());
    }
    // copy the image to dst and wait for the copy (the buffer is reused next time)
    void upload(void* dst, hipStream_t st) {
        hip_check(hipMemcpyAsync(dst, p, size, hipMemcpyHostToDevice, st), "upload");
        hip_check(hipStreamSynchronize(st), "stream synchronize");
    }

private:
    uint8_t*& bref;
    size_t& cref;
};

struct TabOff {
    size_t off = 0, idx = 0, frac = 0;
    PairTable at(char* base) const {
        return PairTable{reinterpret_cast<const int*>(base + off), reinterpret_cast<const int*>(base + idx),
                         reinterpret_cast<const double*>(base + frac)};
    }
};

// ---------------------------------------------------------------------------
// mesh geometry
// ---------------------------------------------------------------------------
struct FaceH {
    int L, R;                    // R < 0: boundary, L is the interior cell
    int bc;
    double nx, ny, area, cx, cy, dLx, dLy, dRx, dRy;
};

// Grow-only pinned host buffer (device-to-host copies of the unique masks).
struct PinnedBuf {
    uint8_t* p = nullptr;
    size_t cap = 0;
    uint8_t* ensure(size_t n) {
        if (n > cap) {
            // pinning is slow: grow geometrically, from 4 MiB
            const size_t want = std::max(n, std::max(2 * cap, (size_t)4 << 20));
            if (p) (void)hipHostFree(p);
            p = nullptr;
            cap = 0;
            hip_check(hipHostMalloc((void**)&p, want, hipHostMallocDefault), "pinned alloc");
            cap = want;
        }
        return p;
    }
    ~PinnedBuf() { if (p) (void)hipHostFree(p); }
};

struct MeshH {
    int ni = 0, nj = 0, dim = 2, n_cells = 0;
    bool per_i = false, per_j = false;
    bool unstructured = false;         // polygons: slots are local edges, slopes by least squares
    std::vector<double> vol, xc, yc;
    std::vector<FaceH> faces;          // interior faces
    std::vector<FaceH> bfaces;         // boundary faces (outward normal)
    std::vector<int> face_of_cell;     // [c][4]: interior face id or -1 (W, E, S, N)
    std::vector<int> bface_of_cell;    // [c][4]: boundary face id or -1
    std::vector<int> nbr;              // [c][4]
    std::vector<CellGeom> geom;
    double hmin = 1e300;
    // Traversal order of the streaming stages: cells tile by tile (tw x th
    // cells, row-major inside a tile and over tiles), so that the cells a
    // stretch of consecutive work items touches, stencils included, stay in one
    // XCD's L2.  order[k] is the k-th cell, rank its inverse.
    std::vector<int> order, rank;
    std::vector<int> face_order, bface_order;   // faces and boundary faces by the rank of their left cell
    // the slot (0..3) of each interior face in its left and right cell, and of
    // each boundary face in its cell (filled on first use; topology only)
    std::vector<int8_t> face_kL, face_kR, bface_k;
};

void finish_order(MeshH& M);

// Tiled traversal order of an ni x nj structured mesh (tw = 0: row-major).
void tile_order(MeshH& M, int tw, int th) {
    const int ni = M.ni, nj = M.nj;
    M.order.clear();
    M.order.reserve(M.n_cells);
    if (tw <= 0 || th <= 0) {
        for (int c = 0; c < M.n_cells; ++c) M.order.push_back(c);
    } else {
        for (int tj = 0; tj < nj; tj += th)
            for (int ti = 0; ti < ni; ti += tw)
                for (int j = tj; j < std::min(nj, tj + th); ++j)
                    for (int i = ti; i < std::min(ni, ti + tw); ++i) M.order.push_back(i + ni * j);
    }
    finish_order(M);
}

// rank and face orders from M.order
void finish_order(MeshH& M) {
    M.rank.assign(M.n_cells, 0);
    for (int k = 0; k < M.n_cells; ++k) M.rank[M.order[k]] = k;
    auto by_rank = [&M](const std::vector<FaceH>& fs, std::vector<int>& out) {
        out.resize(fs.size());
        for (size_t f = 0; f < fs.size(); ++f) out[f] = (int)f;
        std::stable_sort(out.begin(), out.end(), [&](int a, int b) { return M.rank[fs[a].L] < M.rank[fs[b].L]; });
    };
    by_rank(M.faces, M.face_order);
    by_rank(M.bfaces, M.bface_order);
}

void build_mesh(MeshH& M, const mlvs_mesh& in, int dim) {
    const int ni = in.ni, nj = in.nj;
    M.ni = ni; M.nj = nj; M.dim = dim; M.n_cells = ni * nj;
    M.per_i = in.periodic_i != 0; M.per_j = in.periodic_j != 0;
    auto X = [&](int i, int j) { return in.node_x[(size_t)j * (ni + 1) + i]; };
    auto Y = [&](int i, int j) { return in.node_y[(size_t)j * (ni + 1) + i]; };
    const int n = M.n_cells;
    M.vol.resize(n); M.xc.resize(n); M.yc.resize(n);
    for (int j = 0; j < nj; ++j)
        for (int i = 0; i < ni; ++i) {
            const double px[4] = {X(i, j), X(i + 1, j), X(i + 1, j + 1), X(i, j + 1)};
            const double py[4] = {Y(i, j), Y(i + 1, j), Y(i + 1, j + 1), Y(i, j + 1)};
            double a = 0, cx = 0, cy = 0;
            for (int k = 0; k < 4; ++k) {
                const double x0 = px[k], y0 = py[k], x1 = px[(k + 1) % 4], y1 = py[(k + 1) % 4];
                const double cr = x0 * y1 - x1 * y0;
                a += cr; cx += (x0 + x1) * cr; cy += (y0 + y1) * cr;
            }
            a *= 0.5;
            if (!(a > 0)) fail(MLVS_E_ARG, "cell (%d, %d) is not counter-clockwise", i, j);
            const int c = i + ni * j;
            M.vol[c] = a; M.xc[c] = cx / (6.0 * a); M.yc[c] = cy / (6.0 * a);
        }
    double Tix = 0, Tiy = 0, Tjx = 0, Tjy = 0;
    if (M.per_i) { Tix = X(ni, 0) - X(0, 0); Tiy = Y(ni, 0) - Y(0, 0); }
    if (M.per_j) { Tjx = X(0, nj) - X(0, 0); Tjy = Y(0, nj) - Y(0, 0); }
    M.face_of_cell.assign(4 * n, -1);
    M.bface_of_cell.assign(4 * n, -1);
    auto geomf = [](double x0, double y0, double x1, double y1, bool plus_i, FaceH& f) {
        const double tx = x1 - x0, ty = y1 - y0;
        f.area = std::hypot(tx, ty);
        if (plus_i) { f.nx = ty / f.area; f.ny = -tx / f.area; }
        else { f.nx = -ty / f.area; f.ny = tx / f.area; }
        f.cx = 0.5 * (x0 + x1); f.cy = 0.5 * (y0 + y1);
    };
    for (int j = 0; j < nj; ++j)
        for (int i = 0; i < ni + (M.per_i ? 0 : 1); ++i) {
            FaceH f{};
            geomf(X(i, j), Y(i, j), X(i, j + 1), Y(i, j + 1), true, f);
            if ((i > 0 && i < ni) || M.per_i) {
                f.L = (i - 1 + ni) % ni + ni * j;
                f.R = i + ni * j;
                const bool wrap = M.per_i && i == 0;
                f.dLx = f.cx - (M.xc[f.L] - (wrap ? Tix : 0.0));
                f.dLy = f.cy - (M.yc[f.L] - (wrap ? Tiy : 0.0));
                f.dRx = f.cx - M.xc[f.R];
                f.dRy = f.cy - M.yc[f.R];
                f.bc = -1;
                M.faces.push_back(f);
                M.face_of_cell[4 * f.L + 1] = (int)M.faces.size() - 1;
                M.face_of_cell[4 * f.R + 0] = (int)M.faces.size() - 1;
            } else {
                const int c = (i == 0) ? ni * j : ni - 1 + ni * j;
                f.L = c; f.R = -1;
                f.bc = (i == 0) ? in.bc_imin[j] : in.bc_imax[j];
                if (i == 0) { f.nx = -f.nx; f.ny = -f.ny; }
                f.dLx = f.cx - M.xc[c]; f.dLy = f.cy - M.yc[c];
                M.bfaces.push_back(f);
                M.bface_of_cell[4 * c + (i == 0 ? 0 : 1)] = (int)M.bfaces.size() - 1;
            }
        }
    if (dim == 2) {
        for (int j = 0; j < nj + (M.per_j ? 0 : 1); ++j)
            for (int i = 0; i < ni; ++i) {
                FaceH f{};
                geomf(X(i, j), Y(i, j), X(i + 1, j), Y(i + 1, j), false, f);
                if ((j > 0 && j < nj) || M.per_j) {
                    f.L = i + ni * ((j - 1 + nj) % nj);
                    f.R = i + ni * j;
                    const bool wrap = M.per_j && j == 0;
                    f.dLx = f.cx - (M.xc[f.L] - (wrap ? Tjx : 0.0));
                    f.dLy = f.cy - (M.yc[f.L] - (wrap ? Tjy : 0.0));
                    f.dRx = f.cx - M.xc[f.R];
                    f.dRy = f.cy - M.yc[f.R];
                    f.bc = -1;
                    M.faces.push_back(f);
                    M.face_of_cell[4 * f.L + 3] = (int)M.faces.size() - 1;
                    M.face_of_cell[4 * f.R + 2] = (int)M.faces.size() - 1;
                } else {
                    const int c = (j == 0) ? i : i + ni * (nj - 1);
                    f.L = c; f.R = -1;
                    f.bc = (j == 0) ? in.bc_jmin[i] : in.bc_jmax[i];
                    if (j == 0) { f.nx = -f.nx; f.ny = -f.ny; }
                    f.dLx = f.cx - M.xc[c]; f.dLy = f.cy - M.yc[c];
                    M.bfaces.push_back(f);
                    M.bface_of_cell[4 * c + (j == 0 ? 2 : 3)] = (int)M.bfaces.size() - 1;
                }
            }
    }
    for (auto& f : M.bfaces)
        if (f.bc < 0 || f.bc >= in.n_bc) fail(MLVS_E_ARG, "boundary id %d out of range", f.bc);
    // neighbours, direction vectors, spacing
    M.nbr.assign(4 * n, -1);
    M.geom.resize(n);
    for (int c = 0; c < n; ++c) {
        double cenx[4], ceny[4];
        bool have[4] = {false, false, false, false};
        CellGeom& g = M.geom[c];
        g.vol = M.vol[c];
        for (int k = 0; k < 4; ++k) {
            g.dist[k] = 1.0;
            const int f = M.face_of_cell[4 * c + k];
            const int b = M.bface_of_cell[4 * c + k];
            if (f >= 0) {
                const FaceH& F = M.faces[f];
                const bool isL = (F.L == c) && (k == 1 || k == 3);
                const double dx = isL ? F.dLx : F.dRx, dy = isL ? F.dLy : F.dRy;
                cenx[k] = M.xc[c] + dx; ceny[k] = M.yc[c] + dy;
                have[k] = true;
                // neighbour offset: x_n - x_c = (x_f - x_c) - (x_f - x_n)
                const double ox = isL ? (F.dLx - F.dRx) : (F.dRx - F.dLx);
                const double oy = isL ? (F.dLy - F.dRy) : (F.dRy - F.dLy);
                M.nbr[4 * c + k] = isL ? F.R : F.L;
                g.dist[k] = std::hypot(ox, oy);
            } else if (b >= 0) {
                cenx[k] = M.bfaces[b].cx; ceny[k] = M.bfaces[b].cy;
                have[k] = true;
            }
        }
        for (int k = 0; k < 4; ++k) g.inv_dist[k] = 1.0 / g.dist[k];
        double tix = cenx[1] - cenx[0], tiy = ceny[1] - ceny[0];
        double nn = std::hypot(tix, tiy);
        tix /= nn; tiy /= nn;
        double tjx = 0.0, tjy = 1.0;
        if (dim == 2) {
            tjx = cenx[3] - cenx[2]; tjy = ceny[3] - ceny[2];
            nn = std::hypot(tjx, tjy);
            tjx /= nn; tjy /= nn;
        }
        const double det = tix * tjy - tiy * tjx;
        g.G[0] = tjy / det; g.G[1] = -tiy / det; g.G[2] = -tjx / det; g.G[3] = tix / det;
        for (int k = 0; k < 4; ++k)
            if (have[k]) M.hmin = std::min(M.hmin, 2.0 * std::hypot(cenx[k] - M.xc[c], ceny[k] - M.yc[c]));
    }
}

// Unstructured mesh (triangles and quadrilaterals).  Slot k of a cell is its
// k-th edge (node k to node k+1).  An edge shared by two cells is an interior
// face whose left cell is the one met first in cell order, with that cell's
// outward normal; an edge of one cell is a boundary face and must be listed
// with its boundary id.  Slopes: least squares over the face neighbours (a
// boundary face adds a zero-gradient ghost at x_c + 2 (x_f - x_c)), limited by
// Venkatakrishnan's function at every face centre, eps^2 = |V|^(3/2) times the
// square of the stencil's largest |phi| (applied in the kernels).
void build_umesh(MeshH& M, const mlvs_umesh& in) {
    const int n = in.n_cells;
    M.unstructured = true;
    M.dim = 2; M.n_cells = n; M.ni = n; M.nj = 1;
    M.vol.resize(n); M.xc.resize(n); M.yc.resize(n);
    M.face_of_cell.assign(4 * n, -1);
    M.bface_of_cell.assign(4 * n, -1);
    auto node = [&](int v) {
        if (v < 0 || v >= in.n_nodes) fail(MLVS_E_ARG, "node id %d out of range", v);
        return std::make_pair(in.node_x[v], in.node_y[v]);
    };
    std::vector<int> nedge(n);
    for (int c = 0; c < n; ++c) {
        const int b = in.cell_ptr[c], e = in.cell_ptr[c + 1];
        if (e - b != 3 && e - b != 4) fail(MLVS_E_ARG, "cell %d has %d nodes (3 or 4 supported)", c, e - b);
        nedge[c] = e - b;
        double a = 0, cx = 0, cy = 0;
        for (int k = 0; k < e - b; ++k) {
            const auto p0 = node(in.cell_node[b + k]), p1 = node(in.cell_node[b + (k + 1) % (e - b)]);
            const double cr = p0.first * p1.second - p1.first * p0.second;
            a += cr; cx += (p0.first + p1.first) * cr; cy += (p0.second + p1.second) * cr;
        }
        a *= 0.5;
        if (!(a > 0)) fail(MLVS_E_ARG, "cell %d is not counter-clockwise", c);
        M.vol[c] = a; M.xc[c] = cx / (6.0 * a); M.yc[c] = cy / (6.0 * a);
    }
    std::map<std::pair<int, int>, int> bid;
    for (int k = 0; k < in.n_bedges; ++k) {
        const int a = in.bedge[3 * k], b = in.bedge[3 * k + 1];
        bid[std::make_pair(std::min(a, b), std::max(a, b))] = in.bedge[3 * k + 2];
    }
    // pair the edges: first owner -> (cell, slot)
    std::map<std::pair<int, int>, std::pair<int, int>> open;
    std::vector<std::array<int, 4>> fslot;        // interior face: L, kL, R, kR
    for (int c = 0; c < n; ++c) {
        const int b = in.cell_ptr[c], ne = nedge[c];
        for (int k = 0; k < ne; ++k) {
            const int v0 = in.cell_node[b + k], v1 = in.cell_node[b + (k + 1) % ne];
            const auto key = std::make_pair(std::min(v0, v1), std::max(v0, v1));
            if (v0 == v1) fail(MLVS_E_ARG, "cell %d has a repeated node", c);
            auto it = open.find(key);
            if (it == open.end()) {
                open[key] = std::make_pair(c, k);
            } else {
                if (it->second.first < 0) fail(MLVS_E_ARG, "edge (%d, %d) is shared by more than two cells", v0, v1);
                fslot.push_back({it->second.first, it->second.second, c, k});
                it->second.first = -1;
            }
        }
    }
    auto edge_geom = [&](int c, int k, FaceH& f) {
        const int b = in.cell_ptr[c], ne = nedge[c];
        const auto p0 = node(in.cell_node[b + k]), p1 = node(in.cell_node[b + (k + 1) % ne]);
        const double tx = p1.first - p0.first, ty = p1.second - p0.second;
        f.area = std::hypot(tx, ty);
        f.nx = ty / f.area; f.ny = -tx / f.area;        // outward for a counter-clockwise polygon
        f.cx = 0.5 * (p0.first + p1.first); f.cy = 0.5 * (p0.second + p1.second);
    };
    std::sort(fslot.begin(), fslot.end());            // by left cell, then slot
    for (auto& q : fslot) {
        FaceH f{};
        edge_geom(q[0], q[1], f);
        f.L = q[0]; f.R = q[2]; f.bc = -1;
        f.dLx = f.cx - M.xc[f.L]; f.dLy = f.cy - M.yc[f.L];
        f.dRx = f.cx - M.xc[f.R]; f.dRy = f.cy - M.yc[f.R];
        M.faces.push_back(f);
        M.face_of_cell[4 * q[0] + q[1]] = (int)M.faces.size() - 1;
        M.face_of_cell[4 * q[2] + q[3]] = (int)M.faces.size() - 1;
    }
    std::vector<std::pair<int, int>> bslot;
    for (auto& kv : open)
        if (kv.second.first >= 0) bslot.push_back(kv.second);
    std::sort(bslot.begin(), bslot.end());
    for (auto& q : bslot) {
        const int b = in.cell_ptr[q.first], ne = nedge[q.first];
        const int v0 = in.cell_node[b + q.second], v1 = in.cell_node[b + (q.second + 1) % ne];
        auto it = bid.find(std::make_pair(std::min(v0, v1), std::max(v0, v1)));
        if (it == bid.end()) fail(MLVS_E_ARG, "edge (%d, %d) has one cell and no boundary id", v0, v1);
        FaceH f{};
        edge_geom(q.first, q.second, f);
        f.L = q.first; f.R = -1; f.bc = it->second;
        f.dLx = f.cx - M.xc[f.L]; f.dLy = f.cy - M.yc[f.L];
        if (f.bc < 0 || f.bc >= in.n_bc) fail(MLVS_E_ARG, "boundary id %d out of range", f.bc);
        M.bfaces.push_back(f);
        M.bface_of_cell[4 * q.first + q.second] = (int)M.bfaces.size() - 1;
    }
    // neighbours, least-squares coefficients, limiter geometry
    M.nbr.assign(4 * n, -1);
    M.geom.assign(n, CellGeom{});
    for (int c = 0; c < n; ++c) {
        CellGeom& g = M.geom[c];
        g.vol = M.vol[c];
        double ox[4] = {0, 0, 0, 0}, oy[4] = {0, 0, 0, 0};    // least-squares offsets
        bool inner[4] = {false, false, false, false};
        double A00 = 0, A01 = 0, A11 = 0;
        for (int k = 0; k < 4; ++k) {
            g.G[k] = 0.0; g.dist[k] = 1.0; g.inv_dist[k] = 1.0;
            const int f = M.face_of_cell[4 * c + k], b = M.bface_of_cell[4 * c + k];
            if (f >= 0) {
                const FaceH& F = M.faces[f];
                const bool isL = F.L == c;
                g.fox[k] = isL ? F.dLx : F.dRx; g.foy[k] = isL ? F.dLy : F.dRy;
                const int nb = isL ? F.R : F.L;
                M.nbr[4 * c + k] = nb;
                ox[k] = M.xc[nb] - M.xc[c]; oy[k] = M.yc[nb] - M.yc[c];
                inner[k] = true;
                g.dist[k] = std::hypot(ox[k], oy[k]); g.inv_dist[k] = 1.0 / g.dist[k];
            } else if (b >= 0) {
                g.fox[k] = M.bfaces[b].dLx; g.foy[k] = M.bfaces[b].dLy;
                ox[k] = 2.0 * g.fox[k]; oy[k] = 2.0 * g.foy[k];
            } else {
                continue;
            }
            A00 += ox[k] * ox[k]; A01 += ox[k] * oy[k]; A11 += oy[k] * oy[k];
            M.hmin = std::min(M.hmin, 2.0 * std::hypot(g.fox[k], g.foy[k]));
        }
        const double det = A00 * A11 - A01 * A01;
        if (!(det > 0)) fail(MLVS_E_ARG, "cell %d: singular least-squares matrix", c);
        for (int k = 0; k < 4; ++k) {
            g.lx[k] = inner[k] ? (A11 * ox[k] - A01 * oy[k]) / det : 0.0;
            g.ly[k] = inner[k] ? (-A01 * ox[k] + A00 * oy[k]) / det : 0.0;
        }
        const double h = std::sqrt(M.vol[c]);
        g.eps2 = h * h * h;
    }
    // traversal order: Morton order of the cell centroids
    double x0 = 1e300, x1 = -1e300, y0 = 1e300, y1 = -1e300;
    for (int c = 0; c < n; ++c) {
        x0 = std::min(x0, M.xc[c]); x1 = std::max(x1, M.xc[c]);
        y0 = std::min(y0, M.yc[c]); y1 = std::max(y1, M.yc[c]);
    }
    const double span = std::max(std::max(x1 - x0, y1 - y0), 1e-300);
    std::vector<std::pair<uint64_t, int>> key(n);
    for (int c = 0; c < n; ++c) {
        const uint32_t qx = (uint32_t)std::min(65535.0, std::floor((M.xc[c] - x0) / span * 65535.0));
        const uint32_t qy = (uint32_t)std::min(65535.0, std::floor((M.yc[c] - y0) / span * 65535.0));
        uint64_t z = 0;
        for (int bit = 0; bit < 16; ++bit)
            z |= (uint64_t)((qx >> bit) & 1u) << (2 * bit) | (uint64_t)((qy >> bit) & 1u) << (2 * bit + 1);
        key[c] = std::make_pair(z, c);
    }
    std::sort(key.begin(), key.end());
    M.order.resize(n);
    for (int k = 0; k < n; ++k) M.order[k] = key[k].second;
    finish_order(M);
}

}  // namespace

// ---------------------------------------------------------------------------
// the context
// ---------------------------------------------------------------------------
struct mlvs_ctx_s {
    mlvs_physics phys{};
    Phys ph{};
    int prec = 64;
    bool adaptive = false;
    mlvs_adapt_params ap{};
    hipStream_t st = nullptr;
    DevMem dm;
    MeshH mesh;
    Base base;
    std::vector<mlvs_bc> bcs;
    std::vector<std::unique_ptr<Level>> levels;      // representative levels
    std::vector<std::unique_ptr<Level>> ifaces;      // interface levels (no cells)
    std::vector<int> cell_level, cell_slot;
    int64_t step_count = 0;
    int64_t n_cross = 0;
    // device copies
    int *d_cell_lev = nullptr, *d_cell_slot = nullptr, *d_cell_nbr = nullptr, *d_cell_frow = nullptr;
    int* d_order = nullptr;            // the mesh's traversal order (MeshH::order)
    CellGeom* d_geom = nullptr;
    double* d_params = nullptr;
    double* d_cmom = nullptr;          // [chunks][n_cells][NMOM] raw moments of the stored state
    uint8_t* stage_items = nullptr;    // pinned staging areas (Stage) of the work lists and of level installs
    size_t stage_items_cap = 0;
    uint8_t* stage_install = nullptr;
    size_t stage_install_cap = 0;
    void* levels_block = nullptr;      // device block with the current levels' geometry
    double* d_fmom = nullptr;          // [chunks][faces + boundary faces][NFMOM] face moments
    int chunk = 1024;                  // velocity points per chunk (multiple of 64), set per level set
    int chunk_env = 0;                 // MLVS_CHUNK: a fixed chunk instead of the chosen one
    int nch = 1;                       // chunks of the largest level
    double* d_fpar = nullptr;          // [faces + boundary faces][NFP] face records
    bool mom_valid = false;            // d_cmom matches the stored state
    BCDev* d_bcs = nullptr;
    LevelDesc* d_lv = nullptr;
    FaceItem* d_faces = nullptr; int n_faces = 0;    // interior same-level faces, then boundary faces
    int n_bfaces = 0;
    GhostItem* d_ghosts = nullptr; int n_ghosts = 0;
    XFaceItem* d_xfaces = nullptr; int n_xfaces = 0;
    std::vector<DevTable> tables;                    // owned by the current level set
    std::vector<void*> item_allocs;                  // rebuilt with the level set
    double* d_scratch = nullptr; size_t scratch_n = 0;
    unsigned long long* d_neg = nullptr;
    bool state_ready = false;
    // criterion inputs: base grid and per-level maps / masks
    double *d_bx = nullptr, *d_by = nullptr, *d_bw = nullptr, *d_axes = nullptr;
    int *d_ptb_all = nullptr, *d_ptb_off = nullptr;
    double* d_ptab_all = nullptr;      // per level point: criterion tables (Level::crit_tab), levels in order
    int* d_ptab_off = nullptr;         // first point of each level in d_ptab_all
    double* d_ctab = nullptr;          // criterion tables of the base grid's blocks
    // host geometry of recently built levels by their mask (levels recur from
    // one adaptation to the next); copies carry no device memory
    // built levels by mask (host tables only), least recently used evicted
    struct CachedLevel {
        std::unique_ptr<Level> L;
        uint64_t used = 0;
    };
    std::map<std::vector<uint8_t>, CachedLevel> level_cache;
    uint64_t level_tick = 0;
    PinnedBuf pin_masks;               // host copy of the unique masks (adaptation)
    uint8_t* d_kappa_all = nullptr;
    uint8_t* d_kcell = nullptr;
    unsigned long long* d_hash = nullptr;
    int64_t last_unique = 0;
    // learned selector
    int* d_nbr_cell = nullptr;
    float* d_sel = nullptr;
    int sel_K = 0;
    int64_t last_fallback = 0;
    // step graph: the launches of one step captured once per level set
    bool use_graph = false;
    int variant[10] = {1, 1, 1, 1, 1, 1, 1, 1, 1, 0};   // per stage launch variant (autotuned)
    // persistent step (mlvs_set_persistent): one launch per step over the work
    // lists of a device-resident StepArgs, rewritten in place by every level
    // install, so the captured step survives adaptations
    bool persistent = false;
    int tile_w = 0, tile_h = 0;        // traversal tiles of a structured mesh (mlvs_set_tiling)
    StepArgs* d_args = nullptr;
    unsigned int* d_sync = nullptr;    // [0] barrier arrivals, [1] sticky error flag
    int persistent_grid = 0;
    int64_t n_captures = 0, n_graph_launches = 0;
    // Fused step (every level fits one velocity chunk): reconstruction and
    // target in one launch, and the update carries the next step's cell stage.
    bool fuse_allowed = true;          // MLVS_FUSE=0 turns the fused step off
    bool fused = false;
    bool prep_valid = false;           // phi_bar+ rows and parameters match the stored state
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    // cross-level faces run on a second stream (default priority) beside the
    // same-level face stages, forked after the ghost rows and joined before the
    // update
    hipStream_t side_st = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // strict mode (mlvs_set_strict): bit 1 checks the state after every step,
    // bit 2 turns new positivity violations into errors
    int strict = 0;
    unsigned long long* d_check = nullptr;   // [0] cells that failed, [1] smallest such cell
    // selector training data recorded by mlvs_selector_snapshot (host):
    // features [n][10], criterion labels [n], and the catalogue they refer to
    std::vector<float> snap_X;
    std::vector<int32_t> snap_Y;
    std::vector<uint8_t> snap_cat;
    bool sel_on = false;               // learned adaptation enabled
    // counters
    double cnt_updates = 0.0, cnt_iface = 0.0;
    int64_t cnt_adapt = 0;
    double step_points = 0.0, step_iface_points = 0.0;   // per step, current level set

    size_t elt() const { return prec == 32 ? 4 : 8; }
};

namespace {

// (xi_x, xi_y) pairs rounded to float: the FP32 form's reconstruction and
// phi_bar+ rows read one 8-byte pair per point instead of two doubles.
std::vector<float> xy_pairs(const Level& L) {
    std::vector<float> v(2 * (size_t)L.N);
    for (int i = 0; i < L.N; ++i) { v[2 * i] = (float)L.xi_x[i]; v[2 * i + 1] = (float)L.xi_y[i]; }
    return v;
}

void upload_level_geometry(mlvs_ctx c, Level& L) {
    L.d_xy = upload(c->dm, xy_pairs(L), c->st);
    L.d_x = upload(c->dm, L.xi_x, c->st);
    L.d_y = upload(c->dm, L.xi_y, c->st);
    L.d_w = upload(c->dm, L.w, c->st);
    L.d_pt_of_base = upload(c->dm, L.pt_of_base, c->st);
    L.stride = (L.N + 63) / 64 * 64;
}

void free_level(mlvs_ctx c, Level& L) {
    if (!L.geo_in_arena)
        for (void* p : {(void*)L.d_x, (void*)L.d_y, (void*)L.d_w, (void*)L.d_xy, (void*)L.d_pt_of_base})
            c->dm.release(p);
    for (void* p : {L.g, L.h, L.fg, L.fh, L.Fg, L.Fh}) c->dm.release(p);
    L.d_x = L.d_y = L.d_w = nullptr;
    L.d_xy = nullptr;
    L.d_pt_of_base = nullptr;
    L.g = L.h = L.fg = L.fh = L.Fg = L.Fh = nullptr;
}

void alloc_state(mlvs_ctx c, Level& L) {
    const size_t n = (size_t)std::max(L.n_cells, 1) * L.stride * c->elt();
    L.g = c->dm.alloc(n);
    L.h = c->dm.alloc(n);
}


void drop_graph(mlvs_ctx c) {
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->gexec = nullptr;
    c->graph = nullptr;
}

void free_items(mlvs_ctx c) {
    // the persistent step reads its work lists through d_args: its captured
    // graph stays valid; the staged step's launches name the lists directly
    if (!c->persistent) drop_graph(c);
    for (auto& t : c->tables) {
        c->dm.release(t.off);
        c->dm.release(t.idx);
        c->dm.release(t.frac);
    }
    c->tables.clear();
    for (void* p : c->item_allocs) c->dm.release(p);
    c->item_allocs.clear();
    for (auto& L : c->ifaces) free_level(c, *L);
    c->ifaces.clear();
    c->d_faces = nullptr; c->d_fmom = nullptr; c->d_fpar = nullptr; c->d_cmom = nullptr; c->d_ghosts = nullptr; c->d_xfaces = nullptr;
    c->d_lv = nullptr;
    c->n_faces = c->n_bfaces = c->n_ghosts = c->n_xfaces = 0;
}


// Interface level min(kA, kB): host tables only; build_items stages its
// device geometry.
Level* find_iface(mlvs_ctx c, const std::vector<uint8_t>& k, int& idx) {
    for (size_t i = 0; i < c->ifaces.size(); ++i)
        if (c->ifaces[i]->kappa == k) { idx = (int)(c->levels.size() + i); return c->ifaces[i].get(); }
    auto L = level_of_mask(c, k);
    L->is_iface = true;
    L->stride = (L->N + 63) / 64 * 64;
    c->ifaces.push_back(std::move(L));
    idx = (int)(c->levels.size() + c->ifaces.size() - 1);
    return c->ifaces.back().get();
}

Level& level_by_index(mlvs_ctx c, int i) {
    if (i < (int)c->levels.size()) return *c->levels[i];
    return *c->ifaces[i - c->levels.size()];
}

constexpr size_t LEVEL_CACHE_MAX = 256;

// Make room for `add` more levels: drop the least recently used.
void level_cache_trim(mlvs_ctx c, size_t add) {
    while (!c->level_cache.empty() && c->level_cache.size() + add > LEVEL_CACHE_MAX) {
        auto old = c->level_cache.begin();
        for (auto it = c->level_cache.begin(); it != c->level_cache.end(); ++it)
            if (it->second.used < old->second.used) old = it;
        c->level_cache.erase(old);
    }
}

std::unique_ptr<Level> level_of_mask(mlvs_ctx c, const std::vector<uint8_t>& kappa) {
    auto it = c->level_cache.find(kappa);
    if (it == c->level_cache.end()) {
        level_cache_trim(c, 1);
        it = c->level_cache.emplace(kappa, mlvs_ctx_s::CachedLevel{build_level(c->base, kappa), 0}).first;
    }
    it->second.used = ++c->level_tick;
    return std::make_unique<Level>(*it->second.L);
}

// Build the levels of the masks the cache does not hold yet, in parallel on
// the host pool (a level is a pure function of the base grid and its mask),
// so that the level_of_mask calls that follow find them.
void prefill_levels(mlvs_ctx c, const std::vector<std::vector<uint8_t>>& masks) {
    std::vector<const std::vector<uint8_t>*> miss;
    for (auto& k : masks) {
        auto hit = c->level_cache.find(k);
        if (hit != c->level_cache.end()) {
            hit->second.used = ++c->level_tick;          // in use: not the one to evict
            continue;
        }
        bool dup = false;
        for (auto* m : miss) dup = dup || *m == k;
        if (!dup) miss.push_back(&k);
    }
    if (miss.empty()) return;
    level_cache_trim(c, miss.size());
    std::vector<std::unique_ptr<Level>> built(miss.size());
    const std::function<void(int)> job = [&](int t) {
        HostPool& P = HostPool::get();
        for (size_t i = t; i < miss.size(); i += (size_t)std::min<int>(P.size(), (int)miss.size()))
            built[i] = build_level(c->base, *miss[i]);
    };
    HostPool::get().run(std::min<int>(HostPool::get().size(), (int)miss.size()), job);
    for (size_t i = 0; i < miss.size(); ++i)
        c->level_cache.emplace(*miss[i], mlvs_ctx_s::CachedLevel{std::move(built[i]), ++c->level_tick});
}

// The dst <- src tables of a list of level pairs, built in parallel.
std::vector<HostTable> make_tables(const std::vector<std::pair<const Level*, const Level*>>& pairs) {
    std::vector<HostTable> out(pairs.size());
    if (pairs.empty()) return out;
    const int nt = std::min<int>(HostPool::get().size(), (int)pairs.size());
    const std::function<void(int)> job = [&](int t) {
        for (size_t i = t; i < pairs.size(); i += (size_t)nt) out[i] = make_table(*pairs[i].first, *pairs[i].second);
    };
    HostPool::get().run(nt, job);
    return out;
}

// The persistent step's device-resident arguments: the current work lists,
// buffers and counts, written in place (stream-ordered, outside any capture).
void update_step_args(mlvs_ctx c) {
    if (!c->d_args) return;
    StepArgs A{};
    A.lvs = c->d_lv;
    A.ghosts = c->d_ghosts;
    A.faces = c->d_faces;
    A.xfaces = c->d_xfaces;
    A.order = c->d_order;
    A.cell_lev = c->d_cell_lev;
    A.cell_slot = c->d_cell_slot;
    A.cell_nbr = c->d_cell_nbr;
    A.cell_frow = c->d_cell_frow;
    A.geom = c->d_geom;
    A.bcs = c->d_bcs;
    A.params = c->d_params;
    A.cmom = c->d_cmom;
    A.fpar = c->d_fpar;
    A.neg = c->d_neg;
    A.sync = c->d_sync;
    A.n_ghosts = c->n_ghosts;
    A.n_faces = c->n_faces + c->n_bfaces;
    A.n_xfaces = c->n_xfaces;
    A.n_cells = c->mesh.n_cells;
    hip_check(hipMemcpyAsync(c->d_args, &A, sizeof A, hipMemcpyHostToDevice, c->st), "step args upload");
    hip_check(hipStreamSynchronize(c->st), "stream synchronize");
}

// Build face/ghost/cross-face work lists, flux rows and per-cell codes for the
// current level set and upload them (one staged block).  Level state buffers
// must exist.
void build_items(mlvs_ctx c) {
    Marks mk;
    free_items(c);
    mk.mark("items: free", c->st);
    MeshH& M = c->mesh;
    const int n = M.n_cells;
    const int K = (int)c->levels.size();
    Stage stg(c->stage_items, c->stage_items_cap);
    std::vector<int> rows(K, 0), ghosts(K, 0);
    std::vector<int> cell_frow(4 * n, -1);
    std::vector<int> cell_nbr(4 * n, -1);
    std::vector<GhostItem> gitems;
    std::vector<TabOff> gtab;
    std::vector<int> ghost_of((size_t)n * std::max(K, 1), -1);   // [source cell][dst level] -> row
    std::map<std::pair<int, int>, TabOff> tab_of;       // (dst level idx, src level idx)
    auto table = [&](int dst, int src) {
        auto key = std::make_pair(dst, src);
        auto it = tab_of.find(key);
        if (it != tab_of.end()) return it->second;
        const HostTable ht = make_table(level_by_index(c, dst), level_by_index(c, src));
        TabOff t;
        t.off = stg.put(ht.off);
        t.idx = stg.put(ht.idx);
        t.frac = stg.put(ht.frac);
        tab_of[key] = t;
        return t;
    };
    // face codes read by the update: 4 x + 2 final + neg, x = face item (final = 0)
    // or the level row of a final cross-level flux (final = 1)
    auto face_code = [](int x, bool final_flux, bool neg) { return 4 * x + (final_flux ? 2 : 0) + (neg ? 1 : 0); };
    // neighbour codes and ghost rows
    for (int cc = 0; cc < n; ++cc)
        for (int k = 0; k < 4; ++k) {
            const int nb = M.nbr[4 * cc + k];
            if (nb < 0) continue;
            const int lc = c->cell_level[cc], ln = c->cell_level[nb];
            if (lc == ln) { cell_nbr[4 * cc + k] = nb; continue; }
            int& row = ghost_of[(size_t)nb * K + lc];
            if (row < 0) {
                row = ghosts[lc]++;
                GhostItem G{};
                G.n = nb; G.dst = lc; G.row = row;
                gitems.push_back(G);
            }
            cell_nbr[4 * cc + k] = -2 - row;
        }
    {
        // the ghost rows' (dst, src) level tables, built in parallel
        std::vector<std::pair<int, int>> want;
        std::vector<char> seen((size_t)std::max(K * K, 1), 0);
        for (const GhostItem& G : gitems) {
            const int src = c->cell_level[G.n];
            if (!seen[(size_t)G.dst * K + src]) {
                seen[(size_t)G.dst * K + src] = 1;
                want.emplace_back(G.dst, src);
            }
        }
        std::vector<std::pair<const Level*, const Level*>> lp;
        for (auto& ds : want) lp.emplace_back(c->levels[ds.first].get(), c->levels[ds.second].get());
        const std::vector<HostTable> built = make_tables(lp);
        for (size_t i = 0; i < want.size(); ++i) {
            TabOff t;
            t.off = stg.put(built[i].off);
            t.idx = stg.put(built[i].idx);
            t.frac = stg.put(built[i].frac);
            tab_of[want[i]] = t;
        }
        gtab.reserve(gitems.size());
        for (const GhostItem& G : gitems) gtab.push_back(table(G.dst, c->cell_level[G.n]));
    }
    mk.mark("items: ghosts", c->st);
    // face slots of the mesh (topology only, computed once)
    if (M.face_kL.size() != M.faces.size() || M.bface_k.size() != M.bfaces.size()) {
        M.face_kL.assign(M.faces.size(), -1);
        M.face_kR.assign(M.faces.size(), -1);
        for (size_t f = 0; f < M.faces.size(); ++f) {
            const FaceH& F = M.faces[f];
            for (int k = 0; k < 4; ++k) {
                // (a periodic mesh one cell wide has a face twice in one cell:
                // then E/N is the left side, W/S the right one)
                if (M.face_of_cell[4 * F.L + k] == (int)f && (M.unstructured || k == 1 || k == 3)) M.face_kL[f] = (int8_t)k;
                if (M.face_of_cell[4 * F.R + k] == (int)f && (M.unstructured || k == 0 || k == 2)) M.face_kR[f] = (int8_t)k;
            }
        }
        M.bface_k.assign(M.bfaces.size(), -1);
        for (size_t b = 0; b < M.bfaces.size(); ++b)
            for (int k = 0; k < 4; ++k)
                if (M.bface_of_cell[4 * M.bfaces[b].L + k] == (int)b) M.bface_k[b] = (int8_t)k;
    }
    // Interior faces in the traversal order of their left cells.  Two passes
    // over contiguous ranges of that order on the host pool: the first counts,
    // per range, same-level faces, cross-level faces, rows per level and cross
    // faces per level pair; prefix sums over the ranges then give every range
    // its starting indices, and the second pass writes the items in place.
    // The lists, rows and codes are those of one sequential pass.
    const int NF = (int)M.face_order.size();
    const int KK = K * K;
    HostPool& pool = HostPool::get();
    const int NT = std::max(1, std::min(pool.size(), NF / 8192));
    struct RangeCount {
        int same = 0, cross = 0;
        std::vector<int> rows, pair, first;
    };
    std::vector<RangeCount> rc(NT);
    auto range_of = [&](int t, int& lo, int& hi) {
        lo = (int)((long)NF * t / NT);
        hi = (int)((long)NF * (t + 1) / NT);
    };
    {
        const std::function<void(int)> count = [&](int t) {
            RangeCount& r = rc[t];
            r.rows.assign(K, 0);
            r.pair.assign(KK, 0);
            r.first.assign(KK, INT_MAX);
            int lo, hi;
            range_of(t, lo, hi);
            for (int q = lo; q < hi; ++q) {
                const FaceH& F = M.faces[M.face_order[q]];
                const int lL = c->cell_level[F.L], lR = c->cell_level[F.R];
                if (lL == lR) {
                    ++r.same;
                    ++r.rows[lL];
                } else {
                    ++r.cross;
                    ++r.rows[lL];
                    ++r.rows[lR];
                    const int pk = std::min(lL, lR) * K + std::max(lL, lR);
                    if (r.pair[pk]++ == 0) r.first[pk] = q;
                }
            }
        };
        pool.run(NT, count);
    }
    mk.mark("items: faces (count)", c->st);
    // interface levels, created in the order of their first cross face
    std::vector<int> pair_iface(KK, -1), pair_first(KK, INT_MAX);
    for (int t = 0; t < NT; ++t)
        for (int pk = 0; pk < KK; ++pk) pair_first[pk] = std::min(pair_first[pk], rc[t].first[pk]);
    std::vector<int> pairs;
    for (int pk = 0; pk < KK; ++pk)
        if (pair_first[pk] != INT_MAX) pairs.push_back(pk);
    std::sort(pairs.begin(), pairs.end(), [&](int a, int b) { return pair_first[a] < pair_first[b]; });
    std::vector<std::vector<uint8_t>> pair_mask(pairs.size(), std::vector<uint8_t>(c->base.Nb));
    for (size_t i = 0; i < pairs.size(); ++i) {
        const auto& kA = c->levels[pairs[i] / K]->kappa;
        const auto& kB = c->levels[pairs[i] % K]->kappa;
        for (int b = 0; b < c->base.Nb; ++b) pair_mask[i][b] = std::min(kA[b], kB[b]);
    }
    prefill_levels(c, pair_mask);
    for (size_t i = 0; i < pairs.size(); ++i) {
        int iidx = -1;
        find_iface(c, pair_mask[i], iidx);
        pair_iface[pairs[i]] = iidx;
    }
    const int NI = (int)c->ifaces.size();
    mk.mark("items: faces (interface levels)", c->st);
    // starting indices of every range
    struct RangeStart {
        int same = 0, cross = 0;
        std::vector<int> rows, scratch;
    };
    std::vector<RangeStart> st0(NT);
    int n_same = 0, n_cross = 0;
    std::vector<int> scratch_tot(NI, 0);
    for (int t = 0; t < NT; ++t) {
        st0[t].same = n_same;
        st0[t].cross = n_cross;
        st0[t].rows = rows;
        st0[t].scratch = scratch_tot;
        n_same += rc[t].same;
        n_cross += rc[t].cross;
        for (int l = 0; l < K; ++l) rows[l] += rc[t].rows[l];
        for (int pk : pairs) scratch_tot[pair_iface[pk] - K] += rc[t].pair[pk];
    }
    for (int i = 0; i < NI; ++i) c->ifaces[i]->n_rows = scratch_tot[i];
    const int n_bf = (int)M.bface_order.size();
    const int nF_all = n_same + n_bf;
    // cross-level face tables, one set per level pair
    std::vector<std::array<TabOff, 4>> pair_tab(KK);
    {
        std::vector<std::pair<int, int>> want;           // (dst, src) level indices not staged yet
        for (int pk : pairs) {
            const int a = pk / K, b = pk % K, I = pair_iface[pk];
            for (auto ds : {std::make_pair(I, a), std::make_pair(I, b), std::make_pair(a, I), std::make_pair(b, I)})
                if (!tab_of.count(ds) && std::find(want.begin(), want.end(), ds) == want.end()) want.push_back(ds);
        }
        std::vector<std::pair<const Level*, const Level*>> lp;
        for (auto& ds : want) lp.emplace_back(&level_by_index(c, ds.first), &level_by_index(c, ds.second));
        const std::vector<HostTable> built = make_tables(lp);
        for (size_t i = 0; i < want.size(); ++i) {
            TabOff t;
            t.off = stg.put(built[i].off);
            t.idx = stg.put(built[i].idx);
            t.frac = stg.put(built[i].frac);
            tab_of[want[i]] = t;
        }
        for (int pk : pairs) {
            const int a = pk / K, b = pk % K, I = pair_iface[pk];
            pair_tab[pk] = {table(I, a), table(I, b), table(a, I), table(b, I)};
        }
    }
    mk.mark("items: faces (cross-face tables)", c->st);
    // the face items go straight into the staged block
    const size_t o_faces = stg.put(nullptr, sizeof(FaceItem) * (size_t)nF_all);
    FaceItem* fitems = reinterpret_cast<FaceItem*>(stg.p + o_faces);
    std::vector<XFaceItem> xitems(n_cross);
    std::vector<int> xpair(n_cross);
    {
        const std::function<void(int)> fill = [&](int t) {
            int same = st0[t].same, cross = st0[t].cross;
            std::vector<int> row = st0[t].rows, scr = st0[t].scratch;
            int lo, hi;
            range_of(t, lo, hi);
            for (int q = lo; q < hi; ++q) {
                const int f = M.face_order[q];
                const FaceH& F = M.faces[f];
                const int lL = c->cell_level[F.L], lR = c->cell_level[F.R];
                const int kL = M.face_kL[f], kR = M.face_kR[f];
                if (lL == lR) {
                    FaceItem& it = fitems[same];
                    it.L = F.L; it.R = F.R; it.lev = lL; it.row = row[lL]++;
                    it.nx = F.nx; it.ny = F.ny; it.area = F.area;
                    it.dLx = F.dLx; it.dLy = F.dLy; it.dRx = F.dRx; it.dRy = F.dRy;
                    cell_frow[4 * F.L + kL] = face_code(same, false, false);
                    cell_frow[4 * F.R + kR] = face_code(same, false, true);
                    ++same;
                } else {
                    const int pk = std::min(lL, lR) * K + std::max(lL, lR);
                    XFaceItem it{};
                    it.L = F.L; it.R = F.R; it.levA = lL; it.levB = lR;
                    it.rowA = row[lL]++;
                    it.rowB = row[lR]++;
                    it.nx = F.nx; it.ny = F.ny; it.area = F.area;
                    it.dLx = F.dLx; it.dLy = F.dLy; it.dRx = F.dRx; it.dRy = F.dRy;
                    it.levI = pair_iface[pk];
                    it.scratch = scr[pair_iface[pk] - K]++;
                    cell_frow[4 * F.L + kL] = face_code(it.rowA, true, false);
                    cell_frow[4 * F.R + kR] = face_code(it.rowB, true, true);
                    xpair[cross] = pk;
                    xitems[cross++] = it;
                }
            }
        };
        pool.run(NT, fill);
    }
    mk.mark("items: faces (fill)", c->st);
    c->n_cross = n_cross;
    c->step_points = 0.0;
    for (int cc = 0; cc < n; ++cc) c->step_points += c->levels[c->cell_level[cc]]->N;
    c->step_iface_points = 0.0;
    for (auto& it : xitems) c->step_iface_points += level_by_index(c, it.levI).N;
    for (int q = 0; q < n_bf; ++q) {
        const int b = M.bface_order[q];
        const FaceH& F = M.bfaces[b];
        const int lc = c->cell_level[F.L];
        FaceItem it{};
        it.L = F.L; it.R = -1 - F.bc; it.lev = lc; it.row = rows[lc]++;
        it.nx = F.nx; it.ny = F.ny; it.area = F.area; it.dLx = F.dLx; it.dLy = F.dLy;
        cell_frow[4 * F.L + M.bface_k[b]] = face_code(n_same + q, false, false);
        reinterpret_cast<FaceItem*>(stg.p + o_faces)[n_same + q] = it;
    }
    mk.mark("items: host lists", c->st);
    // row buffers
    for (int l = 0; l < K; ++l) {
        Level& L = *c->levels[l];
        L.n_rows = rows[l];
        L.n_ghost = ghosts[l];
        c->dm.release(L.Fg); c->dm.release(L.Fh); c->dm.release(L.fg); c->dm.release(L.fh);
        const size_t nr = (size_t)std::max(L.n_rows, 1) * L.stride * c->elt();
        const size_t nf = (size_t)std::max(L.n_cells + L.n_ghost, 1) * L.stride * c->elt();
        L.Fg = c->dm.alloc(nr); L.Fh = c->dm.alloc(nr);
        L.fg = c->dm.alloc(nf); L.fh = c->dm.alloc(nf);
    }
    struct GeoOff { size_t x, y, w, ptb, xy; };
    std::vector<GeoOff> igeo;
    for (auto& Lp : c->ifaces) {
        Level& L = *Lp;
        const size_t nr = (size_t)std::max(L.n_rows, 1) * L.stride * c->elt();
        L.Fg = c->dm.alloc(nr); L.Fh = c->dm.alloc(nr);
        igeo.push_back({stg.put(L.xi_x), stg.put(L.xi_y), stg.put(L.w), stg.put(L.pt_of_base),
                        stg.put(xy_pairs(L))});
    }
    mk.mark("items: row buffers", c->st);
    c->n_faces = n_same;
    c->n_bfaces = n_bf;
    std::vector<int> ptb, poff, toff;
    std::vector<double> ptab;
    std::vector<uint8_t> kap;
    if (c->base.Nb > 0) {
        for (int l = 0; l < K; ++l) {
            poff.push_back((int)ptb.size());
            ptb.insert(ptb.end(), c->levels[l]->pt_of_base.begin(), c->levels[l]->pt_of_base.end());
            toff.push_back((int)(ptab.size() / 6));
            ptab.insert(ptab.end(), c->levels[l]->crit_tab.begin(), c->levels[l]->crit_tab.end());
            kap.insert(kap.end(), c->levels[l]->kappa.begin(), c->levels[l]->kappa.end());
        }
    }
    // places of the arrays that hold device pointers (filled once the block exists)
    const size_t o_lv = stg.put(nullptr, sizeof(LevelDesc) * (K + c->ifaces.size()));
    const size_t o_gh = stg.put(nullptr, sizeof(GhostItem) * gitems.size());
    const size_t o_xf = stg.put(nullptr, sizeof(XFaceItem) * xitems.size());
    const size_t o_frow = stg.put(cell_frow);
    const size_t o_nbr = stg.put(cell_nbr);
    const size_t o_lev = stg.put(c->cell_level);
    const size_t o_slot = stg.put(c->cell_slot);
    const size_t o_order = stg.put(M.order);
    const size_t o_ptb = stg.put(ptb), o_poff = stg.put(poff), o_kap = stg.put(kap), o_ptab = stg.put(ptab),
                 o_toff = stg.put(toff);
    char* base = static_cast<char*>(c->dm.alloc(stg.size));
    c->item_allocs.push_back(base);
    for (size_t i = 0; i < c->ifaces.size(); ++i) {
        Level& L = *c->ifaces[i];
        L.d_x = reinterpret_cast<double*>(base + igeo[i].x);
        L.d_y = reinterpret_cast<double*>(base + igeo[i].y);
        L.d_w = reinterpret_cast<double*>(base + igeo[i].w);
        L.d_pt_of_base = reinterpret_cast<int*>(base + igeo[i].ptb);
        L.d_xy = reinterpret_cast<float*>(base + igeo[i].xy);
        L.geo_in_arena = true;
    }
    for (size_t i = 0; i < gitems.size(); ++i) gitems[i].tab = gtab[i].at(base);
    for (size_t i = 0; i < xitems.size(); ++i) {
        const auto& T = pair_tab[xpair[i]];
        const bool a_first = xitems[i].levA < xitems[i].levB;     // tables are kept per (low, high) pair
        xitems[i].IfromA = (a_first ? T[0] : T[1]).at(base);
        xitems[i].IfromB = (a_first ? T[1] : T[0]).at(base);
        xitems[i].AfromI = (a_first ? T[2] : T[3]).at(base);
        xitems[i].BfromI = (a_first ? T[3] : T[2]).at(base);
    }
    // level descriptors: representative levels then interface levels
    std::vector<LevelDesc> descs;
    for (int i = 0; i < K + (int)c->ifaces.size(); ++i) {
        Level& L = level_by_index(c, i);
        LevelDesc d{};
        d.N = L.N; d.stride = L.stride; d.n_rows_state = L.n_cells;
        d.xi_x = L.d_x; d.xi_y = L.d_y; d.w = L.d_w; d.xy32 = L.d_xy;
        d.g = L.g; d.h = L.h; d.fg = L.fg; d.fh = L.fh; d.Fg = L.Fg; d.Fh = L.Fh;
        std::copy(L.Minv, L.Minv + 16, d.Minv);
        std::copy(L.G6inv, L.G6inv + 36, d.G6inv);
        std::copy(L.B36, L.B36 + 18, d.B36);
        std::copy(L.H3inv, L.H3inv + 9, d.H3inv);
        descs.push_back(d);
    }
    stg.fill(o_lv, descs);
    stg.fill(o_gh, gitems);
    stg.fill(o_xf, xitems);
    mk.mark("items: staging", c->st);
    stg.upload(base, c->st);
    mk.mark("items: upload", c->st);
    c->d_lv = reinterpret_cast<LevelDesc*>(base + o_lv);
    c->d_faces = reinterpret_cast<FaceItem*>(base + o_faces);
    c->d_ghosts = reinterpret_cast<GhostItem*>(base + o_gh); c->n_ghosts = (int)gitems.size();
    c->d_xfaces = reinterpret_cast<XFaceItem*>(base + o_xf); c->n_xfaces = (int)xitems.size();
    c->d_cell_frow = reinterpret_cast<int*>(base + o_frow);
    c->d_cell_nbr = reinterpret_cast<int*>(base + o_nbr);
    c->d_cell_lev = reinterpret_cast<int*>(base + o_lev);
    c->d_cell_slot = reinterpret_cast<int*>(base + o_slot);
    c->d_order = reinterpret_cast<int*>(base + o_order);
    if (c->base.Nb > 0) {
        c->d_ptb_all = reinterpret_cast<int*>(base + o_ptb);
        c->d_ptb_off = reinterpret_cast<int*>(base + o_poff);
        c->d_ptab_all = reinterpret_cast<double*>(base + o_ptab);
        c->d_ptab_off = reinterpret_cast<int*>(base + o_toff);
        c->d_kappa_all = reinterpret_cast<uint8_t*>(base + o_kap);
    }
    int nmax = 1;
    for (int l = 0; l < K; ++l) nmax = std::max(nmax, c->levels[l]->N);
    // Velocity chunk of the streaming stages: whole rows (one item per face
    // and per cell) unless there are too few faces to fill the GPU with
    // waves, then the fewest chunks that do.  Levels of at most
    // FUSE_MAX_POINTS points always take whole rows and the fused step.
    constexpr int FUSE_MAX_POINTS = 1024, MIN_ITEMS = 16384;
    const int nf_all = std::max<int>(nF_all, 1);
    if (c->chunk_env > 0) {
        c->chunk = c->chunk_env;
    } else {
        int parts = 1;
        if (nmax > FUSE_MAX_POINTS && nf_all < MIN_ITEMS)
            parts = std::min((MIN_ITEMS + nf_all - 1) / nf_all, (nmax + 63) / 64);
        c->chunk = ((nmax + parts - 1) / parts + 63) / 64 * 64;
    }
    if (c->persistent) c->chunk = (nmax + 63) / 64 * 64;    // whole rows (the fused bodies)
    c->nch = (nmax + c->chunk - 1) / c->chunk;
    c->fused = c->fuse_allowed && c->nch == 1 && nmax <= FUSE_MAX_POINTS;
    c->d_fmom = static_cast<double*>(
        c->dm.alloc(sizeof(double) * NFMOM * c->nch * (size_t)std::max(nF_all, 1)));
    c->item_allocs.push_back(c->d_fmom);
    c->d_cmom = static_cast<double*>(c->dm.alloc(sizeof(double) * NMOM * c->nch * (size_t)std::max(n, 1)));
    c->item_allocs.push_back(c->d_cmom);
    c->mom_valid = false;
    c->prep_valid = false;
    c->d_fpar = static_cast<double*>(c->dm.alloc(sizeof(double) * NFP * (size_t)std::max(nF_all, 1)));
    c->item_allocs.push_back(c->d_fpar);
    update_step_args(c);                  // last: every pointer it records is allocated
}

void assign_slots(mlvs_ctx c) {
    const int K = (int)c->levels.size();
    std::vector<int> cnt(K, 0);
    c->cell_slot.resize(c->mesh.n_cells);
    for (int k = 0; k < c->mesh.n_cells; ++k) {
        const int cc = c->mesh.order[k];
        c->cell_slot[cc] = cnt[c->cell_level[cc]]++;
    }
    for (int l = 0; l < K; ++l) c->levels[l]->n_cells = cnt[l];
}

void sync(mlvs_ctx c) { hip_check(hipStreamSynchronize(c->st), "stream synchronize"); }

void build_items(mlvs_ctx c);

// After a new traversal order: slots in that order, every level's state rows
// and prepared cell-stage rows gathered to their new slots, the cell-indexed
// moments and parameters kept, so the next step computes exactly what it
// would have computed before (a copy, no arithmetic).
void retile_rows(mlvs_ctx c) {
    const int n = c->mesh.n_cells;
    const std::vector<int> old_slot = c->cell_slot;
    assign_slots(c);
    const int K = (int)c->levels.size();
    std::vector<std::vector<int>> src(K);
    for (int l = 0; l < K; ++l) src[l].assign(c->levels[l]->n_cells, 0);
    for (int cc = 0; cc < n; ++cc) src[c->cell_level[cc]][c->cell_slot[cc]] = old_slot[cc];
    struct Old { void *g, *h, *fg, *fh; };
    std::vector<Old> old(K);
    for (int l = 0; l < K; ++l) {
        Level& L = *c->levels[l];
        old[l] = {L.g, L.h, L.fg, L.fh};
        L.fg = L.fh = nullptr;             // kept here until copied; build_items allocates new rows
        alloc_state(c, L);
    }
    const bool mom = c->mom_valid, prep = c->prep_valid;
    const size_t cm_bytes = sizeof(double) * NMOM * c->nch * (size_t)std::max(n, 1);
    void* cm = nullptr;
    if (mom && c->d_cmom) {
        cm = c->dm.alloc(cm_bytes);
        hip_check(hipMemcpyAsync(cm, c->d_cmom, cm_bytes, hipMemcpyDeviceToDevice, c->st), "D2D");
    }
    const int nch = c->nch;
    build_items(c);
    std::vector<size_t> off(K + 1, 0);
    for (int l = 0; l < K; ++l) off[l + 1] = off[l] + src[l].size();
    int* d_src = static_cast<int*>(c->dm.alloc(sizeof(int) * std::max<size_t>(off[K], 1)));
    std::vector<int> flat;
    flat.reserve(off[K]);
    for (auto& v : src) flat.insert(flat.end(), v.begin(), v.end());
    hip_check(hipMemcpyAsync(d_src, flat.data(), sizeof(int) * flat.size(), hipMemcpyHostToDevice, c->st), "H2D");
    for (int l = 0; l < K; ++l) {
        Level& L = *c->levels[l];
        const int w16 = (int)((size_t)L.stride * c->elt() / 16);
        const int* rows = d_src + off[l];
        hip_check(launch_gather_rows_16(c->st, old[l].g, w16, rows, L.n_cells, L.g), "gather launch");
        hip_check(launch_gather_rows_16(c->st, old[l].h, w16, rows, L.n_cells, L.h), "gather launch");
        if (prep && old[l].fg) {
            hip_check(launch_gather_rows_16(c->st, old[l].fg, w16, rows, L.n_cells, L.fg), "gather launch");
            hip_check(launch_gather_rows_16(c->st, old[l].fh, w16, rows, L.n_cells, L.fh), "gather launch");
        }
    }
    const bool keep_mom = cm && c->nch == nch;
    if (keep_mom) hip_check(hipMemcpyAsync(c->d_cmom, cm, cm_bytes, hipMemcpyDeviceToDevice, c->st), "D2D");
    sync(c);
    for (int l = 0; l < K; ++l)
        for (void* p : {old[l].g, old[l].h, old[l].fg, old[l].fh}) c->dm.release(p);
    c->dm.release(cm);
    c->dm.release(d_src);
    c->mom_valid = keep_mom;
    c->prep_valid = prep && keep_mom;
}

void do_step(mlvs_ctx c);
// The cell stage reads the raw moments of the stored state from d_cmom; the
// update keeps them current.  After any other write of the state they are
// recomputed once, outside the step (and outside a captured step graph).
void ensure_moments(mlvs_ctx c) {
    if (c->mom_valid) return;
    hip_check(launch_raw_moments(c->prec, c->st, c->d_lv, c->d_cell_lev, c->d_cell_slot, c->mesh.n_cells,
                                 c->d_params, c->d_cmom, c->chunk, c->nch), "moments launch");
    c->mom_valid = true;
}
hipError_t launch_stage(mlvs_ctx c, int stage, hipStream_t on = nullptr);
hipError_t launch_step_kernels(mlvs_ctx c);
std::vector<int> step_stages(mlvs_ctx c);

}  // namespace

// ---------------------------------------------------------------------------
// level switching (remap) -- shared by set_levels and adapt
// ---------------------------------------------------------------------------
namespace {

int64_t install_levels(mlvs_ctx c, std::vector<std::unique_ptr<Level>> nl, const std::vector<int>& new_cell_level) {
    const int n = c->mesh.n_cells;
    Marks mk;
    // keep the old level set alive for the remap
    std::vector<std::unique_ptr<Level>> old = std::move(c->levels);
    std::vector<int> old_level = c->cell_level, old_slot = c->cell_slot;
    free_items(c);
    // the remap reads the old levels' state and geometry only: their row
    // buffers go now (a free waits for the device, so none may come while the
    // remap runs)
    for (auto& L : old) {
        for (void* p : {L->fg, L->fh, L->Fg, L->Fh}) c->dm.release(p);
        L->fg = L->fh = L->Fg = L->Fh = nullptr;
    }
    c->levels = std::move(nl);
    c->cell_level = new_cell_level;
    assign_slots(c);
    // one staged block: the new levels' geometry (kept with the level set) and
    // the remap's descriptors, tables and work list
    Stage stg(c->stage_install, c->stage_install_cap);
    struct GeoOff { size_t x, y, w, ptb, xy; };
    std::vector<GeoOff> geo;
    for (auto& L : c->levels) {
        L->stride = (L->N + 63) / 64 * 64;
        geo.push_back({stg.put(L->xi_x), stg.put(L->xi_y), stg.put(L->w), stg.put(L->pt_of_base),
                       stg.put(xy_pairs(*L))});
        alloc_state(c, *L);
    }
    mk.mark("install: free items, state", c->st);
    std::vector<RemapItem> items(n);
    std::map<std::pair<int, int>, TabOff> tabs;
    std::vector<TabOff> item_tab(n);
    std::vector<char> has_tab(n, 0);
    int64_t changed = 0;
    // the (new level, old level) pairs that need a table, built in parallel
    const int Kn = (int)c->levels.size(), Ko = (int)old.size();
    std::vector<char> same_mask((size_t)Kn * Ko), need((size_t)Kn * Ko, 0);
    for (int d = 0; d < Kn; ++d)
        for (int o = 0; o < Ko; ++o) same_mask[(size_t)d * Ko + o] = old[o]->kappa == c->levels[d]->kappa;
    for (int cc = 0; cc < n; ++cc) {
        const size_t k = (size_t)c->cell_level[cc] * Ko + old_level[cc];
        if (!same_mask[k]) need[k] = 1;
    }
    {
        std::vector<std::pair<int, int>> want;
        std::vector<std::pair<const Level*, const Level*>> lp;
        for (int d = 0; d < Kn; ++d)
            for (int o = 0; o < Ko; ++o)
                if (need[(size_t)d * Ko + o]) {
                    want.emplace_back(d, o);
                    lp.emplace_back(c->levels[d].get(), old[o].get());
                }
        const std::vector<HostTable> built = make_tables(lp);
        for (size_t i = 0; i < want.size(); ++i) {
            TabOff t;
            t.off = stg.put(built[i].off);
            t.idx = stg.put(built[i].idx);
            t.frac = stg.put(built[i].frac);
            tabs.emplace(want[i], t);
        }
    }
    for (int cc = 0; cc < n; ++cc) {
        RemapItem& r = items[cc];
        r.c = cc;
        r.src_lev = old_level[cc]; r.src_slot = old_slot[cc];
        r.dst_lev = c->cell_level[cc]; r.dst_slot = c->cell_slot[cc];
        r.tab = PairTable{nullptr, nullptr, nullptr};
        if (same_mask[(size_t)r.dst_lev * Ko + r.src_lev]) continue;
        ++changed;
        item_tab[cc] = tabs.at(std::make_pair(r.dst_lev, r.src_lev));
        has_tab[cc] = 1;
    }
    const size_t o_od = stg.put(nullptr, sizeof(LevelDesc) * old.size());
    const size_t o_nd = stg.put(nullptr, sizeof(LevelDesc) * c->levels.size());
    const size_t o_items = stg.put(nullptr, sizeof(RemapItem) * n);
    char* base = static_cast<char*>(c->dm.alloc(stg.size));
    for (size_t l = 0; l < c->levels.size(); ++l) {
        Level& L = *c->levels[l];
        L.d_x = reinterpret_cast<double*>(base + geo[l].x);
        L.d_y = reinterpret_cast<double*>(base + geo[l].y);
        L.d_w = reinterpret_cast<double*>(base + geo[l].w);
        L.d_pt_of_base = reinterpret_cast<int*>(base + geo[l].ptb);
        L.d_xy = reinterpret_cast<float*>(base + geo[l].xy);
        L.geo_in_arena = true;
    }
    for (int cc = 0; cc < n; ++cc)
        if (has_tab[cc]) items[cc].tab = item_tab[cc].at(base);
    // old descriptors (state only) and new descriptors
    auto descs_of = [&](std::vector<std::unique_ptr<Level>>& ls) {
        std::vector<LevelDesc> d;
        for (auto& Lp : ls) {
            LevelDesc x{};
            x.N = Lp->N; x.stride = Lp->stride; x.xi_x = Lp->d_x; x.xi_y = Lp->d_y; x.w = Lp->d_w;
            x.xy32 = Lp->d_xy;
            x.g = Lp->g; x.h = Lp->h;
            std::copy(Lp->Minv, Lp->Minv + 16, x.Minv);
            std::copy(Lp->G6inv, Lp->G6inv + 36, x.G6inv);
            std::copy(Lp->B36, Lp->B36 + 18, x.B36);
            std::copy(Lp->H3inv, Lp->H3inv + 9, x.H3inv);
            d.push_back(x);
        }
        return d;
    };
    stg.fill(o_od, descs_of(old));
    stg.fill(o_nd, descs_of(c->levels));
    stg.fill(o_items, items);
    stg.upload(base, c->st);
    mk.mark("install: remap tables", c->st);
    hip_check(launch_remap(c->prec, c->st, reinterpret_cast<LevelDesc*>(base + o_od),
                           reinterpret_cast<LevelDesc*>(base + o_nd), reinterpret_cast<RemapItem*>(base + o_items), n,
                           c->ph, c->d_neg), "remap launch");
    mk.mark("install: remap kernel", c->st);
    // The work lists are built on the host while the remap runs: they read
    // the new level set only, and their upload waits for the remap on the
    // stream.  The old state and geometry are freed after both.
    build_items(c);
    sync(c);
    mk.mark("install: build_items", c->st);
    for (auto& L : old) free_level(c, *L);
    c->dm.release(c->levels_block);            // the old level set's geometry block
    c->levels_block = base;
    mk.mark("install: free old levels", c->st);
    c->mom_valid = false;
    c->prep_valid = false;
    return changed;
}

}  // namespace

// ---------------------------------------------------------------------------
// adaptation: device criterion, host grouping (Sec. 3.2), remap
// ---------------------------------------------------------------------------
namespace {

void run_criterion(mlvs_ctx c) {
    const int n = c->mesh.n_cells;
    const int Nb = c->base.Nb;
    if (!c->d_kcell) c->d_kcell = static_cast<uint8_t*>(c->dm.alloc((size_t)n * Nb));
    if (!c->d_hash) c->d_hash = static_cast<unsigned long long*>(c->dm.alloc(sizeof(unsigned long long) * n));
    hip_check(launch_criterion(c->prec, c->st, c->d_lv, c->d_cell_lev, c->d_cell_slot, n, c->d_ptb_all, c->d_ptb_off,
                               c->d_ptab_all, c->d_ptab_off, c->d_kappa_all, c->d_ctab, c->d_axes, c->base.nx,
                               c->base.ny, c->ap.C_split, c->ap.C_merge, c->ap.eps_merge, c->ap.flux_test, c->d_kcell,
                               c->d_hash),
              "criterion launch");
}

// Strict mode: check every cell's state from the raw moments the last update
// (or the moment pass after an outside write) left; `step` numbers the step
// of the current call (-1: the state before the first step).
void strict_check(mlvs_ctx c, int step) {
    const unsigned long long init[2] = {0ull, ~0ull};
    hip_check(hipMemcpyAsync(c->d_check, init, sizeof init, hipMemcpyHostToDevice, c->st), "H2D");
    hip_check(launch_check_state(c->st, c->d_lv, c->d_cell_lev, c->mesh.n_cells, c->ph, c->d_cmom, c->chunk,
                                 c->d_check), "check launch");
    unsigned long long rec[2] = {0, 0};
    hip_check(hipMemcpyAsync(rec, c->d_check, sizeof rec, hipMemcpyDeviceToHost, c->st), "D2H");
    sync(c);
    if (rec[0] == 0) return;
    const int n = c->mesh.n_cells;
    const int cell = (int)rec[1];
    std::vector<double> f(6 * (size_t)n);
    double* d = static_cast<double*>(c->dm.alloc(sizeof(double) * 6 * (size_t)n));
    hip_check(launch_cell_moments(c->prec, c->st, c->d_lv, c->d_cell_lev, c->d_cell_slot, n, c->d_geom, c->ph, d,
                                  nullptr), "moments launch");
    hip_check(hipMemcpyAsync(f.data(), d, sizeof(double) * 6 * (size_t)n, hipMemcpyDeviceToHost, c->st), "D2H");
    sync(c);
    c->dm.release(d);
    if (step < 0)
        fail(MLVS_E_NUMERIC, "strict mode: %llu cells hold a non-finite or non-positive state before the first step "
             "(first: cell %d, rho = %g, T = %g)", rec[0], cell, f[6 * (size_t)cell], f[6 * (size_t)cell + 3]);
    fail(MLVS_E_NUMERIC, "strict mode: %llu cells hold a non-finite or non-positive state after step %d of this call "
         "(first: cell %d, rho = %g, T = %g)", rec[0], step, cell, f[6 * (size_t)cell], f[6 * (size_t)cell + 3]);
}

// Deduplicate the per-cell masks: returns unique masks (row-major), their first
// cell and count, and the unique index of every cell.
void dedupe(mlvs_ctx c, const uint8_t*& uniq, std::vector<int>& first, std::vector<int64_t>& count,
            std::vector<int>& uidx) {
    const int n = c->mesh.n_cells, Nb = c->base.Nb;
    std::vector<unsigned long long> hs(n);
    hip_check(hipMemcpyAsync(hs.data(), c->d_hash, sizeof(unsigned long long) * n, hipMemcpyDeviceToHost, c->st), "D2H");
    sync(c);
    // group the cells by hash in first-occurrence order: an open-addressing
    // table (multiplicative hash, linear probing), doubled when half full
    uidx.assign(n, -1);
    first.clear();
    count.clear();
    int bits = 12;
    std::vector<unsigned long long> key(size_t(1) << bits);
    std::vector<int> val(size_t(1) << bits, -1);
    auto slot_of = [&](unsigned long long k) {
        const size_t mask = (size_t(1) << bits) - 1;
        size_t j = (size_t)((k * 0x9e3779b97f4a7c15ull) >> (64 - bits));
        while (val[j] >= 0 && key[j] != k) j = (j + 1) & mask;
        return j;
    };
    for (int i = 0; i < n; ++i) {
        size_t j = slot_of(hs[i]);
        if (val[j] >= 0) {
            uidx[i] = val[j];
            ++count[val[j]];
            continue;
        }
        const int u = (int)first.size();
        key[j] = hs[i];
        val[j] = u;
        uidx[i] = u;
        first.push_back(i);
        count.push_back(1);
        if (2 * first.size() > val.size()) {      // rehash into twice the size
            ++bits;
            std::vector<unsigned long long> ok = std::move(key);
            std::vector<int> ov = std::move(val);
            key.assign(size_t(1) << bits, 0ull);
            val.assign(size_t(1) << bits, -1);
            for (size_t q = 0; q < ov.size(); ++q)
                if (ov[q] >= 0) {
                    const size_t t = slot_of(ok[q]);
                    key[t] = ok[q];
                    val[t] = ov[q];
                }
        }
    }
    const int U = (int)first.size();
    int* d_rows = upload(c->dm, first, c->st);
    int* d_rep = upload(c->dm, uidx, c->st);
    uint8_t* d_u = static_cast<uint8_t*>(c->dm.alloc((size_t)U * Nb));
    unsigned long long* d_mis = static_cast<unsigned long long*>(c->dm.alloc(8));
    hip_check(hipMemsetAsync(d_mis, 0, 8, c->st), "memset");
    hip_check(launch_gather_rows_u8(c->st, c->d_kcell, Nb, d_rows, U, d_u), "gather");
    hip_check(launch_compare_rows_u8(c->st, c->d_kcell, Nb, d_rep, d_u, n, d_mis), "compare");
    unsigned long long mis = 0;
    uint8_t* hu = c->pin_masks.ensure((size_t)U * Nb);
    hip_check(hipMemcpyAsync(&mis, d_mis, 8, hipMemcpyDeviceToHost, c->st), "D2H");
    hip_check(hipMemcpyAsync(hu, d_u, (size_t)U * Nb, hipMemcpyDeviceToHost, c->st), "D2H");
    uniq = hu;
    sync(c);
    c->dm.release(d_rows); c->dm.release(d_rep); c->dm.release(d_u); c->dm.release(d_mis);
    if (mis != 0) {
        // hash collision: exact deduplication on the host
        std::vector<uint8_t> all((size_t)n * Nb);
        hip_check(hipMemcpyAsync(all.data(), c->d_kcell, all.size(), hipMemcpyDeviceToHost, c->st), "D2H");
        sync(c);
        std::map<std::vector<uint8_t>, int> ex;
        std::vector<uint8_t> un;
        first.clear(); count.clear();
        for (int i = 0; i < n; ++i) {
            std::vector<uint8_t> row(all.begin() + (size_t)i * Nb, all.begin() + (size_t)(i + 1) * Nb);
            auto it = ex.find(row);
            if (it == ex.end()) {
                ex.emplace(row, (int)first.size());
                uidx[i] = (int)first.size();
                first.push_back(i);
                count.push_back(1);
                un.insert(un.end(), row.begin(), row.end());
            } else {
                uidx[i] = it->second;
                ++count[it->second];
            }
        }
        uint8_t* hx = c->pin_masks.ensure(un.size());
        std::copy(un.begin(), un.end(), hx);
        uniq = hx;
    }
}

// Leader clustering of the unique masks (descending frequency, ties by first
// cell), integer graded distance, enclosing mask = elementwise min, identical
// enclosing masks merged.
//
// Each mask joins the nearest centre founded before it in that order (within
// the threshold; a later centre must be strictly nearer, so ties go to the
// lowest id) or founds a new one; centres are their founding masks.  Done as
// one pass per new centre over every later mask (threaded): a mask has then
// been compared with exactly the centres founded before it, in founding
// order, as a mask-by-mask scan compares it.
void cluster(int Nb, double tau, const uint8_t* uniq, const std::vector<int>& first,
             const std::vector<int64_t>& count, std::vector<std::vector<uint8_t>>& reps, std::vector<int>& level_of_u) {
    const int U = (int)first.size();
    std::vector<int> order(U);
    for (int u = 0; u < U; ++u) order[u] = u;
    std::sort(order.begin(), order.end(), [&](int a, int b) {
        if (count[a] != count[b]) return count[a] > count[b];
        return first[a] < first[b];
    });
    const long thr = (long)std::floor(tau * 3.0 * Nb + 1e-9);
    // Distance sum_b |ka_b - kb_b| in blocks of 256 masks (vectorisable), given
    // up as soon as it exceeds cap.
    auto dist_capped = [Nb](const uint8_t* a, const uint8_t* b, long cap) {
        long d = 0;
        for (int b0 = 0; b0 < Nb; b0 += 256) {
            const int b1 = std::min(Nb, b0 + 256);
            int s = 0;
            for (int k = b0; k < b1; ++k) s += std::abs((int)a[k] - (int)b[k]);
            d += s;
            if (d > cap) return d;
        }
        return d;
    };
    std::vector<int> best(U, -1);          // by position in `order`
    std::vector<long> bestd(U, 0);
    std::vector<int> centres;              // founding positions
    int i = 0;
    while (i < U) {
        int j = i;
        while (j < U && best[j] >= 0) ++j;   // positions i..j-1 are final
        if (j == U) break;
        const int cid = (int)centres.size();
        centres.push_back(j);
        best[j] = cid;
        bestd[j] = 0;
        const uint8_t* kc = &uniq[(size_t)order[j] * Nb];
        parallel_ranges(U - j - 1, std::max(64, (1 << 18) / std::max(Nb, 1)), [&](int lo, int hi) {
            for (int k = j + 1 + lo; k < j + 1 + hi; ++k) {
                const long cap = best[k] < 0 ? thr : bestd[k] - 1;
                if (cap < 0) continue;
                const long d = dist_capped(&uniq[(size_t)order[k] * Nb], kc, cap);
                if (d <= cap) { best[k] = cid; bestd[k] = d; }
            }
        });
        i = j + 1;
    }
    // enclosing masks: elementwise min over each cluster's members
    const int K = (int)centres.size();
    std::vector<std::vector<uint8_t>> kmin(K);
    for (int c = 0; c < K; ++c) {
        const uint8_t* kc = &uniq[(size_t)order[centres[c]] * Nb];
        kmin[c].assign(kc, kc + Nb);
    }
    parallel_ranges(Nb, std::max(64, (1 << 18) / std::max(U, 1)), [&](int lo, int hi) {
        for (int k = 0; k < U; ++k) {
            const uint8_t* ku = &uniq[(size_t)order[k] * Nb];
            uint8_t* km = kmin[best[k]].data();
            for (int b = lo; b < hi; ++b) km[b] = std::min(km[b], ku[b]);
        }
    });
    std::vector<int> cl_of_u(U, -1);
    for (int k = 0; k < U; ++k) cl_of_u[order[k]] = best[k];
    std::vector<int> level_of_cl(kmin.size());
    reps.clear();
    for (size_t k = 0; k < kmin.size(); ++k) {
        int found = -1;
        for (size_t l = 0; l < reps.size(); ++l)
            if (reps[l] == kmin[k]) { found = (int)l; break; }
        if (found < 0) { reps.push_back(kmin[k]); found = (int)reps.size() - 1; }
        level_of_cl[k] = found;
    }
    level_of_u.resize(U);
    for (int u = 0; u < U; ++u) level_of_u[u] = level_of_cl[cl_of_u[u]];
}

void adapt_learned(mlvs_ctx c, mlvs_adapt_report* rep);

double ms_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

void adapt_now(mlvs_ctx c, mlvs_adapt_report* rep) {
    sync(c);                  // the timers below cover the adaptation only, not steps still queued
    auto t0 = std::chrono::steady_clock::now();
    run_criterion(c);
    sync(c);
    const double ms_crit = ms_since(t0);
    t0 = std::chrono::steady_clock::now();
    const uint8_t* uniq = nullptr;
    std::vector<int> first, uidx, level_of_u;
    std::vector<int64_t> count;
    dedupe(c, uniq, first, count, uidx);
    const double ms_dedupe = ms_since(t0);
    t0 = std::chrono::steady_clock::now();
    std::vector<std::vector<uint8_t>> reps;
    cluster(c->base.Nb, c->ap.tau_clust, uniq, first, count, reps, level_of_u);
    const double ms_cluster = ms_since(t0);
    t0 = std::chrono::steady_clock::now();
    std::vector<int> cl(c->mesh.n_cells);
    for (int i = 0; i < c->mesh.n_cells; ++i) cl[i] = level_of_u[uidx[i]];
    // the same catalogue in the same order and the same assignment: nothing to
    // remap or rebuild (the captured step stays valid)
    bool same = reps.size() == c->levels.size() && cl == c->cell_level;
    for (size_t l = 0; same && l < reps.size(); ++l) same = reps[l] == c->levels[l]->kappa;
    int64_t changed = 0;
    if (!same) {
        std::vector<std::unique_ptr<Level>> nl;
        prefill_levels(c, reps);
        for (auto& k : reps) nl.push_back(level_of_mask(c, k));
        changed = install_levels(c, std::move(nl), cl);
    }
    const double ms_install = ms_since(t0);
    c->last_unique = (int64_t)first.size();
    ++c->cnt_adapt;
    if (rep) {
        rep->ms_criterion = ms_crit;
        rep->ms_dedupe = ms_dedupe;
        rep->ms_cluster = ms_cluster;
        rep->ms_install = ms_install;
        rep->n_levels = (int)c->levels.size();
        rep->n_unique = c->last_unique;
        rep->n_changed = changed;
        rep->n_cross = c->n_cross;
        double tot = 0.0;
        for (auto& L : c->levels) tot += (double)L->N * L->n_cells;
        rep->nbar = tot / c->mesh.n_cells;
        unsigned long long v = 0;
        hip_check(hipMemcpyAsync(&v, c->d_neg, 8, hipMemcpyDeviceToHost, c->st), "D2H");
        sync(c);
        rep->neg_count = (int64_t)v;
        rep->n_fallback = 0;
    }
}

void compute_features(mlvs_ctx c, float* d_out) {
    const int n = c->mesh.n_cells;
    double* d8 = static_cast<double*>(c->dm.alloc(sizeof(double) * 8 * (size_t)n));
    hip_check(launch_cell_moments(c->prec, c->st, c->d_lv, c->d_cell_lev, c->d_cell_slot, n, c->d_geom, c->ph,
                                  nullptr, nullptr, d8), "moments launch");
    hip_check(launch_features(c->st, d8, c->d_nbr_cell, c->d_geom, n, c->ph.R, c->ph.T_ref, c->ph.mu_ref,
                              c->ph.omega, c->mesh.unstructured ? 1 : 0, d_out), "features launch");
    sync(c);
    c->dm.release(d8);
}

// The catalogue as bytes: the number of levels, then every level's mask.
std::vector<uint8_t> catalogue_key(mlvs_ctx c) {
    std::vector<uint8_t> k(1, (uint8_t)c->levels.size());
    for (auto& L : c->levels) k.insert(k.end(), L->kappa.begin(), L->kappa.end());
    return k;
}

std::vector<int> level_order(mlvs_ctx c) {
    std::vector<int> order(c->levels.size());
    for (size_t l = 0; l < order.size(); ++l) order[l] = (int)l;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return c->levels[a]->N < c->levels[b]->N; });
    return order;
}

// Tail-mass check of the level d_pred[c] proposed for every cell (d_acc[c] = 1
// where accepted), on the context's stream.  Cells go in groups of one level
// and consecutive slots, so a wave reads the level's tables once per group.
void tail_check(mlvs_ctx c, const int* d_pred, int* d_acc) {
    const int n = c->mesh.n_cells, K = (int)c->levels.size();
    std::vector<int> cnt(K, 0);
    for (int cc = 0; cc < n; ++cc) cnt[c->cell_level[cc]]++;
    std::vector<int> start(K + 1, 0);
    for (int l = 0; l < K; ++l) start[l + 1] = start[l] + (cnt[l] + TAIL_GROUP - 1) / TAIL_GROUP * TAIL_GROUP;
    std::vector<int> grp(start[K], -1);
    for (int cc = 0; cc < n; ++cc) grp[start[c->cell_level[cc]] + c->cell_slot[cc]] = cc;
    int* d_grp = upload(c->dm, grp, c->st);
    hip_check(launch_tail_check(c->prec, c->st, c->d_lv, c->d_cell_lev, c->d_cell_slot, d_grp,
                                start[K] / TAIL_GROUP, c->d_ptb_all, c->d_ptb_off, c->d_kappa_all, d_pred, c->d_bw,
                                c->base.nx, c->base.ny, c->ap.C_split, d_acc), "tail check launch");
    sync(c);
    c->dm.release(d_grp);
}

// Frozen catalogue: predicted level per cell, tail-mass check, criterion labels
// for the rejected cells, remap of the cells whose level changes.
void adapt_learned(mlvs_ctx c, mlvs_adapt_report* rep) {
    const int n = c->mesh.n_cells, K = (int)c->levels.size(), Nb = c->base.Nb;
    if (K != c->sel_K) fail(MLVS_E_STATE, "selector trained for %d levels, catalogue has %d", c->sel_K, K);
    float* d_feat = static_cast<float*>(c->dm.alloc(sizeof(float) * 10 * (size_t)n));
    int* d_pred = static_cast<int*>(c->dm.alloc(sizeof(int) * (size_t)n));
    int* d_acc = static_cast<int*>(c->dm.alloc(sizeof(int) * (size_t)n));
    compute_features(c, d_feat);
    hip_check(launch_mlp_predict(c->st, c->d_sel, K, d_feat, n, 1, d_pred, nullptr), "predict launch");
    tail_check(c, d_pred, d_acc);
    std::vector<int> pred(n), acc(n);
    hip_check(hipMemcpyAsync(pred.data(), d_pred, sizeof(int) * n, hipMemcpyDeviceToHost, c->st), "D2H");
    hip_check(hipMemcpyAsync(acc.data(), d_acc, sizeof(int) * n, hipMemcpyDeviceToHost, c->st), "D2H");
    sync(c);
    std::vector<int> rej;
    for (int i = 0; i < n; ++i)
        if (!acc[i]) rej.push_back(i);
    std::vector<int> cl = pred;
    if (!rej.empty()) {
        if (!c->d_kcell) c->d_kcell = static_cast<uint8_t*>(c->dm.alloc((size_t)n * Nb));
        if (!c->d_hash) c->d_hash = static_cast<unsigned long long*>(c->dm.alloc(sizeof(unsigned long long) * n));
        int* d_list = upload(c->dm, rej, c->st);
        hip_check(launch_criterion(c->prec, c->st, c->d_lv, c->d_cell_lev, c->d_cell_slot, (int)rej.size(),
                                   c->d_ptb_all, c->d_ptb_off, c->d_ptab_all, c->d_ptab_off, c->d_kappa_all,
                                   c->d_ctab, c->d_axes, c->base.nx, c->base.ny, c->ap.C_split, c->ap.C_merge,
                                   c->ap.eps_merge,
                                   c->ap.flux_test, c->d_kcell, c->d_hash, d_list), "criterion launch");
        std::vector<int> order = level_order(c);
        int* d_order = upload(c->dm, order, c->st);
        hip_check(launch_labels(c->st, c->d_kcell, n, Nb, c->d_kappa_all, d_order, K, d_pred), "labels launch");
        std::vector<int> lab(n);
        hip_check(hipMemcpyAsync(lab.data(), d_pred, sizeof(int) * n, hipMemcpyDeviceToHost, c->st), "D2H");
        sync(c);
        const int finest = order.back();
        for (int i : rej) cl[i] = lab[i] >= 0 ? lab[i] : finest;
        c->dm.release(d_list);
        c->dm.release(d_order);
    }
    c->dm.release(d_feat);
    c->dm.release(d_pred);
    c->dm.release(d_acc);
    std::vector<std::unique_ptr<Level>> nl;
    for (auto& L : c->levels) nl.push_back(build_level(c->base, L->kappa));
    const int64_t changed = install_levels(c, std::move(nl), cl);
    c->last_fallback = (int64_t)rej.size();
    ++c->cnt_adapt;
    if (rep) {
        rep->n_levels = K;
        rep->n_unique = -1;
        rep->n_changed = changed;
        rep->n_cross = c->n_cross;
        double tot = 0.0;
        for (auto& L : c->levels) tot += (double)L->N * L->n_cells;
        rep->nbar = tot / n;
        unsigned long long v = 0;
        hip_check(hipMemcpyAsync(&v, c->d_neg, 8, hipMemcpyDeviceToHost, c->st), "D2H");
        sync(c);
        rep->neg_count = (int64_t)v;
        rep->n_fallback = c->last_fallback;
    }
}

// Context-free device buffers for the network routines (hipMalloc, null stream).
struct DevBuf {
    void* p = nullptr;
    explicit DevBuf(size_t n) {
        if (hipMalloc(&p, n == 0 ? 8 : n) != hipSuccess) fail(MLVS_E_OOM, "hipMalloc of %zu bytes failed", n);
    }
    ~DevBuf() { if (p) (void)hipFree(p); }
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    template <typename T> T* as() { return static_cast<T*>(p); }
};

void check_mlp_args(int K) {
    if (K < 2 || K > 16) fail(MLVS_E_ARG, "number of classes must be in [2, 16]");
}

}  // namespace

// ---------------------------------------------------------------------------
// ABI
// ---------------------------------------------------------------------------
extern "C" {

mlvs_status mlvs_mlp_nparams(int K, int64_t* n) {
    return guarded([&] {
        check_mlp_args(K);
        if (!n) fail(MLVS_E_ARG, "null output");
        *n = mlp_nparams(K);
    });
}

mlvs_status mlvs_features(mlvs_ctx c, float* out) {
    return guarded([&] {
        if (!c || !out) fail(MLVS_E_ARG, "null argument");
        if (!c->state_ready) fail(MLVS_E_STATE, "state not initialised");
        if (c->phys.dim != 2) fail(MLVS_E_STATE, "features need dim = 2");
        const int n = c->mesh.n_cells;
        float* d = static_cast<float*>(c->dm.alloc(sizeof(float) * 10 * (size_t)n));
        compute_features(c, d);
        hip_check(hipMemcpyAsync(out, d, sizeof(float) * 10 * (size_t)n, hipMemcpyDeviceToHost, c->st), "D2H");
        sync(c);
        c->dm.release(d);
    });
}

mlvs_status mlvs_labels(mlvs_ctx c, int32_t* out) {
    return guarded([&] {
        if (!c || !out) fail(MLVS_E_ARG, "null argument");
        if (!c->adaptive) fail(MLVS_E_STATE, "context was created without adaptation parameters");
        if (!c->state_ready) fail(MLVS_E_STATE, "state not initialised");
        run_criterion(c);
        const int n = c->mesh.n_cells;
        std::vector<int> order = level_order(c);
        int* d_order = upload(c->dm, order, c->st);
        int* d_lab = static_cast<int*>(c->dm.alloc(sizeof(int) * (size_t)n));
        hip_check(launch_labels(c->st, c->d_kcell, n, c->base.Nb, c->d_kappa_all, d_order, (int)order.size(), d_lab),
                  "labels launch");
        hip_check(hipMemcpyAsync(out, d_lab, sizeof(int) * (size_t)n, hipMemcpyDeviceToHost, c->st), "D2H");
        sync(c);
        c->dm.release(d_order);
        c->dm.release(d_lab);
    });
}

mlvs_status mlvs_mlp_eval(const float* params, int K, const float* X, const int32_t* y, int B, float* probs,
                          float* grad, double* loss) {
    return guarded([&] {
        check_mlp_args(K);
        if (!params || !X || !y || B < 1) fail(MLVS_E_ARG, "bad arguments");
        for (int b = 0; b < B; ++b)
            if (y[b] < 0 || y[b] >= K) fail(MLVS_E_ARG, "label out of range");
        const size_t np = mlp_nparams(K), Bs = (size_t)B;
        DevBuf P(4 * np), G(4 * np), Xd(40 * Bs), Yd(4 * Bs), PR(4 * K * Bs), PART(mlp_part_bytes(B, K)), LS(8);
        hip_check(hipMemcpy(P.p, params, 4 * np, hipMemcpyHostToDevice), "H2D");
        hip_check(hipMemcpy(Xd.p, X, 40 * Bs, hipMemcpyHostToDevice), "H2D");
        hip_check(hipMemcpy(Yd.p, y, 4 * Bs, hipMemcpyHostToDevice), "H2D");
        hip_check(launch_mlp_eval(nullptr, P.as<float>(), K, Xd.as<float>(), Yd.as<int>(), B, PR.as<float>(), PART.p,
                                  G.as<float>(), LS.as<double>()), "forward/backward");
        hip_check(hipDeviceSynchronize(), "sync");
        if (probs) hip_check(hipMemcpy(probs, PR.p, 4 * K * Bs, hipMemcpyDeviceToHost), "D2H");
        if (grad) hip_check(hipMemcpy(grad, G.p, 4 * np, hipMemcpyDeviceToHost), "D2H");
        if (loss) {
            double sum = 0.0;
            hip_check(hipMemcpy(&sum, LS.p, 8, hipMemcpyDeviceToHost), "D2H");
            *loss = sum / B;
        }
    });
}

mlvs_status mlvs_mlp_eval_noalloc(const float* d_params, int K, const float* d_X, const int32_t* d_y, int B,
                                  float* d_probs, float* d_grad, double* d_loss_sum, void* stream) {
    return guarded([&] {
        check_mlp_args(K);
        if (!d_params || !d_X || !d_y) fail(MLVS_E_ARG, "null argument");
        if (B < 1 || B > NOALLOC_MAX_BATCH)
            fail(MLVS_E_ARG, "batch of %d samples: this entry point takes 1 to %d", B, NOALLOC_MAX_BATCH);
        hip_check(launch_mlp_eval_noalloc(static_cast<hipStream_t>(stream), d_params, K, d_X, d_y, B, d_probs, d_grad,
                                          d_loss_sum), "forward/backward launch");
    });
}

mlvs_status mlvs_mlp_predict(const float* params, int K, const float* X, int B, int bf16, int32_t* classes,
                             float* probs) {
    return guarded([&] {
        check_mlp_args(K);
        if (!params || !X || !classes || B < 1) fail(MLVS_E_ARG, "bad arguments");
        const size_t np = mlp_nparams(K), Bs = (size_t)B;
        DevBuf P(4 * np), Xd(40 * Bs), C(4 * Bs), PR(4 * K * Bs);
        hip_check(hipMemcpy(P.p, params, 4 * np, hipMemcpyHostToDevice), "H2D");
        hip_check(hipMemcpy(Xd.p, X, 40 * Bs, hipMemcpyHostToDevice), "H2D");
        hip_check(launch_mlp_predict(nullptr, P.as<float>(), K, Xd.as<float>(), B, bf16, C.as<int>(),
                                     probs ? PR.as<float>() : nullptr), "predict");
        hip_check(hipDeviceSynchronize(), "sync");
        hip_check(hipMemcpy(classes, C.p, 4 * Bs, hipMemcpyDeviceToHost), "D2H");
        if (probs) hip_check(hipMemcpy(probs, PR.p, 4 * K * Bs, hipMemcpyDeviceToHost), "D2H");
    });
}

}  // extern "C"

namespace {

// Training loop on the device (FP32 forward/backward/Adam kernels, hipMalloc
// and the null stream): params in/out on the host, samples X [n][10], y [n].
void train_network(float* params, int K, const float* X, const int32_t* y, int64_t n, const mlvs_train_cfg* cfg,
                   mlvs_train_report* rep) {
    {
        check_mlp_args(K);
        if (!params || !X || !y || !cfg || n < 2 || n > (int64_t)1 << 30) fail(MLVS_E_ARG, "bad arguments");
        if (cfg->epochs < 1 || cfg->batch < 1 || !(cfg->val_frac >= 0.0 && cfg->val_frac < 1.0))
            fail(MLVS_E_ARG, "bad training configuration");
        for (int64_t i = 0; i < n; ++i)
            if (y[i] < 0 || y[i] >= K) fail(MLVS_E_ARG, "label out of range at %lld", (long long)i);
        const int64_t n_val = (int64_t)std::floor(cfg->val_frac * n);
        const int64_t n_tr = n - n_val;
        if (n_tr < 1) fail(MLVS_E_ARG, "no training samples");
        const int np = mlp_nparams(K);
        std::vector<float> P(params, params + np);
        for (int k = 0; k < 10; ++k) {   // input standardisation from the training samples
            double m = 0.0, v = 0.0;
            for (int64_t i = 0; i < n_tr; ++i) m += X[i * 10 + k];
            m /= n_tr;
            for (int64_t i = 0; i < n_tr; ++i) v += (X[i * 10 + k] - m) * (X[i * 10 + k] - m);
            v = std::sqrt(v / n_tr);
            P[np - 20 + k] = (float)m;
            P[np - 10 + k] = (float)(v > 1e-12 ? v : 1.0);
        }
        const int B = (int)std::min<int64_t>(cfg->batch, n_tr);
        const size_t ns = (size_t)n;
        DevBuf Pd(4 * (size_t)np), M(4 * (size_t)np), V(4 * (size_t)np), Xd(40 * ns), Yd(4 * ns),
            IDX(4 * (size_t)n_tr), PART(mlp_part_bytes(B, K));
        const int64_t steps_per_epoch = n_tr / B;
        const int64_t total_steps = steps_per_epoch * cfg->epochs;
        DevBuf LS(8 * (size_t)std::max<int64_t>(total_steps, 1));
        hip_check(hipMemcpy(Pd.p, P.data(), 4 * (size_t)np, hipMemcpyHostToDevice), "H2D");
        hip_check(hipMemcpy(Xd.p, X, 40 * ns, hipMemcpyHostToDevice), "H2D");
        hip_check(hipMemcpy(Yd.p, y, 4 * ns, hipMemcpyHostToDevice), "H2D");
        hip_check(hipMemset(M.p, 0, 4 * (size_t)np), "memset");
        hip_check(hipMemset(V.p, 0, 4 * (size_t)np), "memset");
        std::vector<int> perm(n_tr);
        uint64_t state = cfg->seed ? cfg->seed : 0x2545f4914f6cdd1dull;
        auto next = [&]() {   // splitmix64
            uint64_t z = (state += 0x9e3779b97f4a7c15ull);
            z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
            z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
            return z ^ (z >> 31);
        };
        hipEvent_t e0, e1;
        hip_check(hipEventCreate(&e0), "event");
        hip_check(hipEventCreate(&e1), "event");
        hip_check(hipEventRecord(e0, nullptr), "event");
        int64_t t = 0;
        for (int ep = 0; ep < cfg->epochs; ++ep) {
            for (int64_t i = 0; i < n_tr; ++i) perm[i] = (int)i;
            for (int64_t i = n_tr - 1; i > 0; --i) std::swap(perm[i], perm[next() % (uint64_t)(i + 1)]);
            hip_check(hipMemcpy(IDX.p, perm.data(), 4 * (size_t)n_tr, hipMemcpyHostToDevice), "H2D");
            for (int64_t sidx = 0; sidx < steps_per_epoch; ++sidx, ++t) {
                hip_check(launch_mlp_train_step(nullptr, Pd.as<float>(), K, Xd.as<float>(), Yd.as<int>(),
                                                IDX.as<int>() + sidx * B, B, PART.p, LS.as<double>() + t, M.as<float>(),
                                                V.as<float>(), (float)cfg->lr, (float)cfg->beta1, (float)cfg->beta2,
                                                (float)cfg->eps, (int)(t + 1)), "training step");
            }
        }
        hip_check(hipEventRecord(e1, nullptr), "event");
        hip_check(hipEventSynchronize(e1), "event");
        float ms = 0.f;
        hip_check(hipEventElapsedTime(&ms, e0, e1), "elapsed");
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        std::vector<double> ls(std::max<int64_t>(total_steps, 1), 0.0);
        if (total_steps > 0) hip_check(hipMemcpy(ls.data(), LS.p, 8 * total_steps, hipMemcpyDeviceToHost), "D2H");
        hip_check(hipMemcpy(P.data(), Pd.p, 4 * (size_t)np, hipMemcpyDeviceToHost), "D2H");
        std::copy(P.begin(), P.end(), params);
        std::vector<int> cls(n);
        DevBuf C(4 * ns);
        hip_check(launch_mlp_predict(nullptr, Pd.as<float>(), K, Xd.as<float>(), (int)n, 0, C.as<int>(), nullptr),
                  "predict");
        hip_check(hipMemcpy(cls.data(), C.p, 4 * ns, hipMemcpyDeviceToHost), "D2H");
        if (rep) {
            int64_t ok_tr = 0, ok_va = 0;
            for (int64_t i = 0; i < n; ++i) {
                if (i < n_tr) ok_tr += cls[i] == y[i];
                else ok_va += cls[i] == y[i];
            }
            auto mean_epoch = [&](int ep) {
                double sum = 0.0;
                for (int64_t k = 0; k < steps_per_epoch; ++k) sum += ls[ep * steps_per_epoch + k] / B;
                return steps_per_epoch ? sum / steps_per_epoch : 0.0;
            };
            rep->loss_first = mean_epoch(0);
            rep->loss_last = mean_epoch(cfg->epochs - 1);
            rep->train_acc = (double)ok_tr / n_tr;
            rep->val_acc = n_val ? (double)ok_va / n_val : 0.0;
            rep->n_train = n_tr;
            rep->n_val = n_val;
            rep->steps = total_steps;
            rep->ms = ms;
        }
    }
}

// He-normal initial weights (fan-in scaling, zero biases, identity
// standardisation) from a splitmix64 stream and the Box-Muller transform.
std::vector<float> he_init(int K, uint64_t seed) {
    const int np = mlp_nparams(K);
    std::vector<float> P(np, 0.f);
    uint64_t st = seed ^ 0x6a09e667f3bcc909ull;
    auto next = [&]() {
        uint64_t z = (st += 0x9e3779b97f4a7c15ull);
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
        return z ^ (z >> 31);
    };
    auto normal = [&]() {
        const double u1 = ((next() >> 11) + 0.5) * 0x1.0p-53, u2 = (next() >> 11) * 0x1.0p-53;
        return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
    };
    const int H = 64, NF = 10;
    size_t o = 0;
    auto fill = [&](int rows, int fan_in) {
        const double sd = std::sqrt(2.0 / fan_in);
        for (int k = 0; k < rows * fan_in; ++k) P[o++] = (float)(sd * normal());
        o += rows;   // biases stay zero
    };
    fill(H, NF);
    fill(H, H);
    fill(K, H);
    for (int k = 0; k < NF; ++k) P[o + NF + k] = 1.f;   // mean 0, std 1 (set again by training)
    return P;
}

}  // namespace

extern "C" {

mlvs_status mlvs_mlp_train(float* params, int K, const float* X, const int32_t* y, int64_t n,
                           const mlvs_train_cfg* cfg, mlvs_train_report* rep) {
    return guarded([&] { train_network(params, K, X, y, n, cfg, rep); });
}

mlvs_status mlvs_selector_set(mlvs_ctx c, const float* params, int K) {
    return guarded([&] {
        if (!c) fail(MLVS_E_ARG, "null context");
        if (!params) {
            c->dm.release(c->d_sel);
            c->d_sel = nullptr;
            c->sel_K = 0;
            c->sel_on = false;
            return;
        }
        check_mlp_args(K);
        if (!c->adaptive) fail(MLVS_E_STATE, "context was created without adaptation parameters");
        if (K != (int)c->levels.size())
            fail(MLVS_E_ARG, "K = %d but the catalogue has %d levels", K, (int)c->levels.size());
        const int np = mlp_nparams(K);
        c->dm.release(c->d_sel);
        c->d_sel = static_cast<float*>(c->dm.alloc(4 * (size_t)np));
        hip_check(hipMemcpyAsync(c->d_sel, params, 4 * (size_t)np, hipMemcpyHostToDevice, c->st), "H2D");
        sync(c);
        c->sel_K = K;
        c->sel_on = true;
    });
}

mlvs_status mlvs_selector_snapshot(mlvs_ctx c, int reset, int64_t* n_samples) {
    return guarded([&] {
        if (!c) fail(MLVS_E_ARG, "null context");
        if (!c->adaptive) fail(MLVS_E_STATE, "context was created without adaptation parameters");
        if (!c->state_ready) fail(MLVS_E_STATE, "state not initialised");
        if (c->phys.dim != 2) fail(MLVS_E_STATE, "features need dim = 2");
        const std::vector<uint8_t> cat = catalogue_key(c);
        if (reset) {
            c->snap_X.clear();
            c->snap_Y.clear();
            c->snap_cat.clear();
        }
        if (!c->snap_Y.empty() && cat != c->snap_cat)
            fail(MLVS_E_STATE, "the catalogue changed since the first recorded snapshot (reset the store)");
        const int n = c->mesh.n_cells;
        float* d_feat = static_cast<float*>(c->dm.alloc(sizeof(float) * 10 * (size_t)n));
        int* d_lab = static_cast<int*>(c->dm.alloc(sizeof(int) * (size_t)n));
        compute_features(c, d_feat);
        run_criterion(c);
        std::vector<int> order = level_order(c);
        int* d_order = upload(c->dm, order, c->st);
        hip_check(launch_labels(c->st, c->d_kcell, n, c->base.Nb, c->d_kappa_all, d_order, (int)order.size(), d_lab),
                  "labels launch");
        const size_t o = c->snap_Y.size();
        c->snap_X.resize(10 * (o + n));
        c->snap_Y.resize(o + n);
        hip_check(hipMemcpyAsync(c->snap_X.data() + 10 * o, d_feat, sizeof(float) * 10 * (size_t)n,
                                 hipMemcpyDeviceToHost, c->st), "D2H");
        hip_check(hipMemcpyAsync(c->snap_Y.data() + o, d_lab, sizeof(int) * (size_t)n, hipMemcpyDeviceToHost, c->st),
                  "D2H");
        sync(c);
        c->dm.release(d_feat);
        c->dm.release(d_lab);
        c->dm.release(d_order);
        c->snap_cat = cat;
        if (n_samples) *n_samples = (int64_t)c->snap_Y.size();
    });
}

mlvs_status mlvs_selector_train(mlvs_ctx c, const mlvs_train_cfg* cfg, mlvs_train_report* rep) {
    return guarded([&] {
        if (!c || !cfg) fail(MLVS_E_ARG, "null argument");
        if (!c->adaptive) fail(MLVS_E_STATE, "context was created without adaptation parameters");
        if (c->snap_Y.empty()) fail(MLVS_E_STATE, "no snapshots recorded");
        if (catalogue_key(c) != c->snap_cat)
            fail(MLVS_E_STATE, "the catalogue changed since the snapshots were recorded");
        const int K = (int)c->levels.size();
        check_mlp_args(K);
        std::vector<float> X;
        std::vector<int32_t> y;
        X.reserve(c->snap_X.size());
        y.reserve(c->snap_Y.size());
        for (size_t i = 0; i < c->snap_Y.size(); ++i)
            if (c->snap_Y[i] >= 0) {
                y.push_back(c->snap_Y[i]);
                X.insert(X.end(), c->snap_X.begin() + 10 * i, c->snap_X.begin() + 10 * (i + 1));
            }
        std::vector<float> P = he_init(K, cfg->seed);
        train_network(P.data(), K, X.data(), y.data(), (int64_t)y.size(), cfg, rep);
        const int np = mlp_nparams(K);
        c->dm.release(c->d_sel);
        c->d_sel = static_cast<float*>(c->dm.alloc(4 * (size_t)np));
        hip_check(hipMemcpyAsync(c->d_sel, P.data(), 4 * (size_t)np, hipMemcpyHostToDevice, c->st), "H2D");
        sync(c);
        c->sel_K = K;
    });
}

mlvs_status mlvs_selector_enable(mlvs_ctx c, int on) {
    return guarded([&] {
        if (!c || (on != 0 && on != 1)) fail(MLVS_E_ARG, "bad arguments");
        if (on && !c->d_sel) fail(MLVS_E_STATE, "no network installed (mlvs_selector_train or mlvs_selector_set)");
        if (on && c->sel_K != (int)c->levels.size())
            fail(MLVS_E_STATE, "the network has %d classes but the catalogue %d levels", c->sel_K,
                 (int)c->levels.size());
        c->sel_on = on != 0;
    });
}

mlvs_status mlvs_selector_check(mlvs_ctx c, const int32_t* levels, int32_t* accept) {
    return guarded([&] {
        if (!c || !levels || !accept) fail(MLVS_E_ARG, "null argument");
        if (c->ph.D != 2) fail(MLVS_E_STATE, "the tail-mass check needs dim = 2");
        const int n = c->mesh.n_cells, K = (int)c->levels.size();
        std::vector<int> lev(levels, levels + n);
        for (int i = 0; i < n; ++i)
            if (lev[i] < 0 || lev[i] >= K) fail(MLVS_E_ARG, "level %d of cell %d is not in [0, %d)", lev[i], i, K);
        int* d_lev = upload(c->dm, lev, c->st);
        int* d_acc = static_cast<int*>(c->dm.alloc(sizeof(int) * (size_t)n));
        tail_check(c, d_lev, d_acc);
        hip_check(hipMemcpyAsync(accept, d_acc, sizeof(int) * (size_t)n, hipMemcpyDeviceToHost, c->st), "D2H");
        sync(c);
        c->dm.release(d_lev);
        c->dm.release(d_acc);
    });
}

mlvs_status mlvs_selector_params(mlvs_ctx c, float* out, int* K) {
    return guarded([&] {
        if (!c || !K) fail(MLVS_E_ARG, "null argument");
        *K = c->sel_K;
        if (!out || !c->d_sel) return;
        hip_check(hipMemcpyAsync(out, c->d_sel, 4 * (size_t)mlp_nparams(c->sel_K), hipMemcpyDeviceToHost, c->st),
                  "D2H");
        sync(c);
    });
}


const char* mlvs_last_error(void) { return g_last_error.c_str(); }

mlvs_status mlvs_vgrid_newton_cotes(int n, double a, double* x, double* w) {
    return guarded([&] {
        if (!x || !w || !(a > 0)) fail(MLVS_E_ARG, "bad Newton-Cotes arguments");
        newton_cotes(n, a, x, w);
    });
}

mlvs_status mlvs_vgrid_gauss_hermite(int n, double R, double T0, double* x, double* w) {
    return guarded([&] {
        if (!x || !w || !(R > 0) || !(T0 > 0)) fail(MLVS_E_ARG, "bad Gauss-Hermite arguments");
        gauss_hermite(n, R, T0, x, w);
    });
}

mlvs_status mlvs_mu_ref_from_kn(double Kn, double rho, double T, double R, double L, double omega, double* mu) {
    return guarded([&] {
        if (!mu) fail(MLVS_E_ARG, "null output");
        const double cst = 15.0 * std::sqrt(M_PI) / (2.0 * (5.0 - 2.0 * omega) * (7.0 - 2.0 * omega));
        *mu = cst * Kn * rho * std::sqrt(2.0 * R * T) * L;
    });
}

// One of mesh (structured) and umesh (unstructured) is given.
static mlvs_status create_impl(const mlvs_physics* phys, const mlvs_mesh* mesh, const mlvs_umesh* umesh,
                               const mlvs_vgrid* vg, const mlvs_adapt_params* adapt, const mlvs_device* dev,
                               mlvs_ctx* out) {
    mlvs_ctx c = nullptr;
    mlvs_status s = guarded([&] {
        if (!phys || (!mesh && !umesh) || !vg || !out) fail(MLVS_E_ARG, "null argument");
        if (phys->dim != 1 && phys->dim != 2) fail(MLVS_E_ARG, "dim must be 1 or 2");
        if (phys->precision != 32 && phys->precision != 64) fail(MLVS_E_ARG, "precision must be 32 or 64");
        if (phys->compat != 0 && phys->compat != 4 && phys->compat != 8) fail(MLVS_E_ARG, "compat must be 0, 4 or 8");
        if (phys->compat == 8 && phys->dim != 2) fail(MLVS_E_ARG, "compat 8 needs dim = 2");
        if (phys->map_moments != 0 && phys->map_moments != 4 && phys->map_moments != 9)
            fail(MLVS_E_ARG, "map_moments must be 0, 4 or 9");
        if (phys->map_moments == 9 && phys->dim != 2) fail(MLVS_E_ARG, "map_moments 9 needs dim = 2");
        if (phys->positivity != 0 && phys->positivity != 1) fail(MLVS_E_ARG, "positivity must be 0 or 1");
        if (phys->positivity == 1 && phys->map_moments != 4)
            fail(MLVS_E_ARG, "the exponential fallback needs map_moments = 4");
        if (!(phys->R > 0) || !(phys->mu_ref > 0) || !(phys->T_ref > 0)) fail(MLVS_E_ARG, "bad physical constants");
        if (mesh) {
            if (mesh->ni < 1 || mesh->nj < 1 || !mesh->node_x || !mesh->node_y) fail(MLVS_E_ARG, "bad mesh");
            if (phys->dim == 1 && mesh->nj != 1) fail(MLVS_E_ARG, "1-D meshes need nj = 1");
            if ((int64_t)mesh->ni * mesh->nj > (1 << 30)) fail(MLVS_E_ARG, "mesh too large");
        } else {
            if (phys->dim != 2) fail(MLVS_E_ARG, "unstructured meshes need dim = 2");
            if (umesh->n_cells < 1 || umesh->n_nodes < 3 || !umesh->node_x || !umesh->node_y || !umesh->cell_ptr ||
                !umesh->cell_node || (umesh->n_bedges > 0 && !umesh->bedge) || umesh->n_bedges < 0 ||
                (umesh->n_bc > 0 && !umesh->bcs) || umesh->n_bc < 0)
                fail(MLVS_E_ARG, "bad mesh");
            if (umesh->n_cells > (1 << 28)) fail(MLVS_E_ARG, "mesh too large");
            if (umesh->cell_ptr[0] != 0) fail(MLVS_E_ARG, "cell_ptr[0] must be 0");
            for (int k = 0; k < umesh->n_cells; ++k)
                if (umesh->cell_ptr[k + 1] < umesh->cell_ptr[k]) fail(MLVS_E_ARG, "cell_ptr must not decrease");
        }
        if (!vg->x || !vg->wx || vg->nx < 2 || vg->ny < 1 || !vg->y || !vg->wy) fail(MLVS_E_ARG, "bad velocity grid");
        if (phys->dim == 1 && vg->ny != 1) fail(MLVS_E_ARG, "1-D needs ny = 1");
        if (adapt && phys->dim != 2) fail(MLVS_E_ARG, "multi-level velocity spaces need dim = 2");
        if (adapt && (adapt->interval < 0 || adapt->C_merge > adapt->C_split))
            fail(MLVS_E_ARG, "bad adaptation parameters");
        c = new mlvs_ctx_s();
        c->phys = *phys;
        c->prec = phys->precision;
        if (dev) { c->dm.dev = *dev; c->st = (hipStream_t)dev->stream; }
        c->adaptive = adapt != nullptr;
        if (adapt) c->ap = *adapt;
        if (umesh) build_umesh(c->mesh, *umesh);
        else build_mesh(c->mesh, *mesh, phys->dim);
        if (mesh) {
            // traversal tiles (MLVS_TILE=WxH overrides; 0 = row-major)
            int tw = 16, th = 8;
            if (const char* e = std::getenv("MLVS_TILE")) {
                if (std::sscanf(e, "%dx%d", &tw, &th) != 2) tw = th = 0;
                if (tw < 0 || th < 0 || tw > 4096 || th > 4096) fail(MLVS_E_ARG, "bad MLVS_TILE");
            }
            if (phys->dim != 2) tw = th = 0;
            tile_order(c->mesh, tw, th);
            c->tile_w = tw;
            c->tile_h = th;
        }
        if (mesh) c->bcs.assign(mesh->bcs, mesh->bcs + mesh->n_bc);
        else c->bcs.assign(umesh->bcs, umesh->bcs + umesh->n_bc);
        for (auto& b : c->bcs)
            if (b.kind < 1 || b.kind > 3) fail(MLVS_E_ARG, "unknown boundary kind %d", b.kind);
        Base& B = c->base;
        B.nx = vg->nx; B.ny = vg->ny; B.N = B.nx * B.ny;
        B.nbx = B.nx / 2; B.nby = phys->dim == 2 ? B.ny / 2 : 0;
        B.Nb = B.nbx * B.nby;
        double vmax = 0.0;
        for (int iy = 0; iy < B.ny; ++iy)
            for (int ix = 0; ix < B.nx; ++ix) {
                B.x.push_back(vg->x[ix]);
                B.y.push_back(phys->dim == 2 ? vg->y[iy] : 0.0);
                B.w.push_back(vg->wx[ix] * (phys->dim == 2 ? vg->wy[iy] : 1.0));
                vmax = std::max(vmax, std::hypot(B.x.back(), B.y.back()));
            }
        for (int ix = 0; ix < B.nx; ++ix) B.axes.push_back(vg->x[ix]);
        for (int ix = 0; ix < B.nx; ++ix) B.axes.push_back(vg->wx[ix]);
        for (int iy = 0; iy < B.ny; ++iy) B.axes.push_back(phys->dim == 2 ? vg->y[iy] : 0.0);
        for (int iy = 0; iy < B.ny; ++iy) B.axes.push_back(phys->dim == 2 ? vg->wy[iy] : 1.0);
        Phys& ph = c->ph;
        ph.D = phys->dim; ph.K = phys->K; ph.R = phys->R; ph.Pr = phys->Pr; ph.omega = phys->omega;
        ph.mu_ref = phys->mu_ref; ph.T_ref = phys->T_ref;
        ph.dt = phys->dt > 0 ? phys->dt : phys->cfl * c->mesh.hmin / vmax;
        ph.compat = phys->compat; ph.face_compat = phys->face_compat; ph.map_moments = phys->map_moments;
        ph.positivity = phys->positivity;
        ph.mesh_kind = c->mesh.unstructured ? 1 : 0;
        hip_check(hipStreamCreateWithFlags(&c->side_st, hipStreamNonBlocking), "stream create");
        hip_check(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming), "event create");
        hip_check(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming), "event create");
        // device geometry
        c->d_geom = upload(c->dm, c->mesh.geom, c->st);
        c->d_nbr_cell = upload(c->dm, c->mesh.nbr, c->st);
        c->d_bx = upload(c->dm, B.x, c->st);
        c->d_by = upload(c->dm, B.y, c->st);
        c->d_bw = upload(c->dm, B.w, c->st);
        c->d_axes = upload(c->dm, B.axes, c->st);
        block_tables(B);
        c->d_ctab = upload(c->dm, B.ctab, c->st);
        std::vector<BCDev> bd;
        for (auto& b : c->bcs) bd.push_back(BCDev{b.kind, 0, b.rho, b.u, b.v, b.T});
        c->d_bcs = upload(c->dm, bd, c->st);
        c->d_params = static_cast<double*>(c->dm.alloc(sizeof(double) * NPARAM * c->mesh.n_cells));
        hip_check(hipMemsetAsync(c->d_params, 0, sizeof(double) * NPARAM * c->mesh.n_cells, c->st), "memset");
        // counters: [0] positivity violations, [1] exponential fallbacks, [2] failed ones
        c->d_neg = static_cast<unsigned long long*>(c->dm.alloc(24));
        hip_check(hipMemsetAsync(c->d_neg, 0, 24, c->st), "memset");
        c->d_args = static_cast<StepArgs*>(c->dm.alloc(sizeof(StepArgs)));
        c->d_sync = static_cast<unsigned int*>(c->dm.alloc(8));
        hip_check(hipMemsetAsync(c->d_sync, 0, 8, c->st), "memset");
        // velocity chunk of the streaming stages (MLVS_CHUNK overrides; multiple of 64)
        if (const char* e = std::getenv("MLVS_FUSE")) c->fuse_allowed = std::atoi(e) != 0;
        if (const char* e = std::getenv("MLVS_CHUNK")) {
            const int v = std::atoi(e);
            if (v < 64 || v % 64 != 0) fail(MLVS_E_ARG, "MLVS_CHUNK must be a positive multiple of 64");
            c->chunk_env = v;
        }
        // one level: the base grid itself
        std::vector<uint8_t> k0(B.Nb, 0);
        c->levels.push_back(build_level(B, k0));
        c->cell_level.assign(c->mesh.n_cells, 0);
        assign_slots(c);
        upload_level_geometry(c, *c->levels[0]);
        alloc_state(c, *c->levels[0]);
        build_items(c);
        sync(c);
        *out = c;
    });
    if (s != MLVS_OK && c) {
        if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
        if (c->ev_join) (void)hipEventDestroy(c->ev_join);
        if (c->side_st) (void)hipStreamDestroy(c->side_st);
        c->dm.release_all();
        delete c;
    }
    return s;
}

mlvs_status mlvs_create(const mlvs_physics* phys, const mlvs_mesh* mesh, const mlvs_vgrid* vg,
                        const mlvs_adapt_params* adapt, const mlvs_device* dev, mlvs_ctx* out) {
    if (!mesh) return guarded([&] { fail(MLVS_E_ARG, "null argument"); });
    return create_impl(phys, mesh, nullptr, vg, adapt, dev, out);
}

mlvs_status mlvs_create_unstructured(const mlvs_physics* phys, const mlvs_umesh* mesh, const mlvs_vgrid* vg,
                                     const mlvs_adapt_params* adapt, const mlvs_device* dev, mlvs_ctx* out) {
    if (!mesh) return guarded([&] { fail(MLVS_E_ARG, "null argument"); });
    return create_impl(phys, nullptr, mesh, vg, adapt, dev, out);
}

void mlvs_destroy(mlvs_ctx c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->st);
    if (c->side_st) (void)hipStreamSynchronize(c->side_st);
    drop_graph(c);
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    if (c->side_st) (void)hipStreamDestroy(c->side_st);
    c->dm.release_all();
    if (c->stage_items) (void)hipHostFree(c->stage_items);
    if (c->stage_install) (void)hipHostFree(c->stage_install);
    delete c;
}

mlvs_status mlvs_init_equilibrium(mlvs_ctx c, const double* st) {
    return guarded([&] {
        if (!c || !st) fail(MLVS_E_ARG, "null argument");
        for (int i = 0; i < c->mesh.n_cells; ++i)
            if (!(st[4 * i] > 0) || !(st[4 * i + 3] > 0)) fail(MLVS_E_ARG, "non-positive density or temperature at cell %d", i);
        std::vector<double> v(st, st + 4 * (size_t)c->mesh.n_cells);
        double* d = upload(c->dm, v, c->st);
        hip_check(launch_init_eq(c->prec, c->st, c->d_lv, c->d_cell_lev, c->d_cell_slot, c->mesh.n_cells, d, c->ph,
                                 c->d_params), "init launch");
        sync(c);
        c->dm.release(d);
        c->state_ready = true;
        c->mom_valid = false;
    c->prep_valid = false;
        c->step_count = 0;
    });
}

mlvs_status mlvs_step(mlvs_ctx c, int n_steps) {
    return guarded([&] {
        if (!c || n_steps < 0) fail(MLVS_E_ARG, "bad arguments");
        if (!c->state_ready) fail(MLVS_E_STATE, "state not initialised");
        unsigned long long neg0[3] = {0, 0, 0};
        if (c->strict & 2) {
            hip_check(hipMemcpyAsync(neg0, c->d_neg, sizeof neg0, hipMemcpyDeviceToHost, c->st), "D2H");
            sync(c);
        }
        if (c->strict & 1) {
            ensure_moments(c);
            strict_check(c, -1);
        }
        for (int k = 0; k < n_steps; ++k) {
            do_step(c);
            if (c->strict & 1) strict_check(c, k);
        }
        if (c->strict & 2) {
            unsigned long long neg1[3] = {0, 0, 0};
            hip_check(hipMemcpyAsync(neg1, c->d_neg, sizeof neg1, hipMemcpyDeviceToHost, c->st), "D2H");
            sync(c);
            if (neg1[0] != neg0[0] || neg1[2] != neg0[2])
                fail(MLVS_E_NUMERIC,
                     "strict mode: %llu mapping corrections made a nonnegative g negative, %llu exponential "
                     "corrections did not converge during this call",
                     neg1[0] - neg0[0], neg1[2] - neg0[2]);
        }
    });
}

mlvs_status mlvs_set_adapt(mlvs_ctx c, const mlvs_adapt_params* adapt) {
    return guarded([&] {
        if (!c || !adapt) fail(MLVS_E_ARG, "null argument");
        if (!c->adaptive) fail(MLVS_E_STATE, "context was created without adaptation parameters");
        if (adapt->interval < 0 || adapt->C_merge > adapt->C_split || !(adapt->tau_clust >= 0.0))
            fail(MLVS_E_ARG, "bad adaptation parameters");
        c->ap = *adapt;
    });
}

mlvs_status mlvs_set_strict(mlvs_ctx c, int flags) {
    return guarded([&] {
        if (!c || flags < 0 || flags > 3) fail(MLVS_E_ARG, "bad arguments");
        if ((flags & 1) && !c->d_check) c->d_check = static_cast<unsigned long long*>(c->dm.alloc(16));
        c->strict = flags;
    });
}

mlvs_status mlvs_moments(mlvs_ctx c, double* out) {
    return guarded([&] {
        if (!c || !out) fail(MLVS_E_ARG, "null argument");
        if (!c->state_ready) fail(MLVS_E_STATE, "state not initialised");
        const int n = c->mesh.n_cells;
        double* d = static_cast<double*>(c->dm.alloc(sizeof(double) * 6 * n));
        hip_check(launch_cell_moments(c->prec, c->st, c->d_lv, c->d_cell_lev, c->d_cell_slot, n, c->d_geom, c->ph, d,
                                      nullptr), "moments launch");
        hip_check(hipMemcpyAsync(out, d, sizeof(double) * 6 * n, hipMemcpyDeviceToHost, c->st), "D2H");
        sync(c);
        c->dm.release(d);
    });
}

mlvs_status mlvs_stress(mlvs_ctx c, double* out) {
    return guarded([&] {
        if (!c || !out) fail(MLVS_E_ARG, "null argument");
        if (!c->state_ready) fail(MLVS_E_STATE, "state not initialised");
        if (c->ph.D != 2) fail(MLVS_E_STATE, "the stress output needs dim = 2");
        const int n = c->mesh.n_cells;
        double* d = static_cast<double*>(c->dm.alloc(sizeof(double) * 3 * n));
        hip_check(launch_cell_moments(c->prec, c->st, c->d_lv, c->d_cell_lev, c->d_cell_slot, n, c->d_geom, c->ph,
                                      nullptr, nullptr, nullptr, d), "moments launch");
        hip_check(hipMemcpyAsync(out, d, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, c->st), "D2H");
        sync(c);
        c->dm.release(d);
    });
}

mlvs_status mlvs_totals(mlvs_ctx c, double out[4]) {
    return guarded([&] {
        if (!c || !out) fail(MLVS_E_ARG, "null argument");
        if (!c->state_ready) fail(MLVS_E_STATE, "state not initialised");
        const int n = c->mesh.n_cells;
        double* d = static_cast<double*>(c->dm.alloc(sizeof(double) * (4 * (size_t)n + 4)));
        hip_check(launch_cell_moments(c->prec, c->st, c->d_lv, c->d_cell_lev, c->d_cell_slot, n, c->d_geom, c->ph,
                                      nullptr, d), "totals launch");
        hip_check(launch_sum_rows(c->st, d, n, 4, d + 4 * (size_t)n), "sum launch");
        hip_check(hipMemcpyAsync(out, d + 4 * (size_t)n, sizeof(double) * 4, hipMemcpyDeviceToHost, c->st), "D2H");
        sync(c);
        c->dm.release(d);
    });
}

mlvs_status mlvs_info(mlvs_ctx c, double* dt, int64_t* n_cells, int32_t* n_blocks, int32_t* n_base) {
    return guarded([&] {
        if (!c) fail(MLVS_E_ARG, "null context");
        if (dt) *dt = c->ph.dt;
        if (n_cells) *n_cells = c->mesh.n_cells;
        if (n_blocks) *n_blocks = c->base.Nb;
        if (n_base) *n_base = c->base.N;
    });
}

mlvs_status mlvs_variants(int stage, int* count) {
    return guarded([&] {
        if (!count || stage < 0 || stage > 9) fail(MLVS_E_ARG, "bad arguments");
        *count = (stage == 1 || stage == 6) ? 1 : stage == 9 ? persistent_variant_count() : variant_count();
    });
}

mlvs_status mlvs_set_variant(mlvs_ctx c, int stage, int v) {
    return guarded([&] {
        int cnt = 0;
        if (!c || mlvs_variants(stage, &cnt) != MLVS_OK || v < 0 || v >= cnt) fail(MLVS_E_ARG, "bad variant");
        sync(c);
        drop_graph(c);
        c->variant[stage] = v;
    });
}

mlvs_status mlvs_set_persistent(mlvs_ctx c, int on) {
    return guarded([&] {
        if (!c || (on != 0 && on != 1)) fail(MLVS_E_ARG, "bad arguments");
        if (!c->state_ready) fail(MLVS_E_STATE, "state not initialised");
        sync(c);
        if ((on != 0) == c->persistent) return;
        drop_graph(c);
        c->persistent = on != 0;
        build_items(c);               // chunks (whole rows) and the device-resident arguments
    });
}

mlvs_status mlvs_set_tiling(mlvs_ctx c, int tw, int th) {
    return guarded([&] {
        if (!c) fail(MLVS_E_ARG, "null context");
        if (tw < 0 || th < 0 || tw > 4096 || th > 4096 || ((tw == 0) != (th == 0)))
            fail(MLVS_E_ARG, "bad tiles %d x %d", tw, th);
        if (c->mesh.unstructured || c->phys.dim != 2) fail(MLVS_E_STATE, "tiles apply to 2-D structured meshes");
        if (tw == c->tile_w && th == c->tile_h) return;
        tile_order(c->mesh, tw, th);
        c->tile_w = tw;
        c->tile_h = th;
        retile_rows(c);
    });
}

mlvs_status mlvs_tiling(mlvs_ctx c, int* tw, int* th) {
    return guarded([&] {
        if (!c) fail(MLVS_E_ARG, "null context");
        if (tw) *tw = c->tile_w;
        if (th) *th = c->tile_h;
    });
}

mlvs_status mlvs_graph_info(mlvs_ctx c, int* persistent, int64_t* captures, int64_t* launches, int* grid,
                            int* error) {
    return guarded([&] {
        if (!c) fail(MLVS_E_ARG, "null context");
        if (persistent) *persistent = c->persistent ? 1 : 0;
        if (captures) *captures = c->n_captures;
        if (launches) *launches = c->n_graph_launches;
        if (grid) *grid = c->persistent_grid;
        if (error) {
            unsigned int v[2] = {0, 0};
            hip_check(hipMemcpyAsync(v, c->d_sync, sizeof v, hipMemcpyDeviceToHost, c->st), "D2H");
            sync(c);
            *error = (int)v[1];
        }
    });
}

mlvs_status mlvs_set_graph(mlvs_ctx c, int on) {
    return guarded([&] {
        if (!c) fail(MLVS_E_ARG, "null context");
        if (on && c->st == nullptr) fail(MLVS_E_STATE, "graph capture needs a non-default stream");
        sync(c);
        drop_graph(c);
        c->use_graph = on != 0;
    });
}

mlvs_status mlvs_counters(mlvs_ctx c, int64_t* steps, double* cell_updates, double* iface_points,
                          int64_t* adaptations) {
    return guarded([&] {
        if (!c) fail(MLVS_E_ARG, "null context");
        if (steps) *steps = c->step_count;
        if (cell_updates) *cell_updates = c->cnt_updates;
        if (iface_points) *iface_points = c->cnt_iface;
        if (adaptations) *adaptations = c->cnt_adapt;
    });
}

mlvs_status mlvs_time_stage(mlvs_ctx c, int stage, int reps, double* ms) {
    return guarded([&] {
        if (!c || !ms || reps < 1 || stage < 0 || stage > 9) fail(MLVS_E_ARG, "bad arguments");
        if ((stage == 7 || stage == 8) && !c->fused) fail(MLVS_E_STATE, "fused stages need levels of one chunk");
        if (stage == 9 && !c->persistent) fail(MLVS_E_STATE, "the persistent step is off (mlvs_set_persistent)");
        if (!c->state_ready) fail(MLVS_E_STATE, "state not initialised");
        if (stage == 9 && !c->prep_valid) {
            hip_check(launch_stage(c, 0), "cell stage launch");
            c->prep_valid = true;
        }
        if (stage == 6 && !c->adaptive) fail(MLVS_E_STATE, "criterion needs adaptation parameters");
        ensure_moments(c);
        // every stage but the update only rewrites its own outputs; the update
        // advances the state, which is saved here and put back afterwards
        std::vector<std::pair<void*, void*>> saved;    // (live buffer, copy)
        std::vector<size_t> saved_bytes;
        if (stage == 5 || stage == 8 || stage == 9) {
            auto keep = [&](void* p, size_t nb) {
                if (!p || nb == 0) return;
                void* q = c->dm.alloc(nb);
                hip_check(hipMemcpyAsync(q, p, nb, hipMemcpyDeviceToDevice, c->st), "D2D");
                saved.emplace_back(p, q);
                saved_bytes.push_back(nb);
            };
            for (auto& L : c->levels) {
                const size_t nb = (size_t)L->n_cells * L->stride * c->elt();
                keep(L->g, nb);
                keep(L->h, nb);
            }
            keep(c->d_cmom, sizeof(double) * NMOM * c->nch * (size_t)c->mesh.n_cells);
            if (stage == 8 || stage == 9) {   // the next step's cell stage: phi_bar+ rows and parameters
                for (auto& L : c->levels) {
                    const size_t nb = (size_t)L->n_cells * L->stride * c->elt();
                    keep(L->fg, nb);
                    keep(L->fh, nb);
                }
                keep(c->d_params, sizeof(double) * NPARAM * (size_t)c->mesh.n_cells);
            }
        }
        hipEvent_t e0, e1;
        hip_check(hipEventCreate(&e0), "event");
        hip_check(hipEventCreate(&e1), "event");
        double tot = 0.0;
        for (int r = 0; r < reps; ++r) {
            hip_check(hipEventRecord(e0, c->st), "event record");
            if (stage == 6) run_criterion(c);
            else hip_check(launch_stage(c, stage), "stage launch");
            hip_check(hipEventRecord(e1, c->st), "event record");
            hip_check(hipEventSynchronize(e1), "event sync");
            float t = 0.f;
            hip_check(hipEventElapsedTime(&t, e0, e1), "elapsed");
            tot += t;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        for (size_t k = 0; k < saved.size(); ++k) {
            hip_check(hipMemcpyAsync(saved[k].first, saved[k].second, saved_bytes[k], hipMemcpyDeviceToDevice, c->st),
                      "D2D");
        }
        sync(c);
        for (auto& pr : saved) c->dm.release(pr.second);
        *ms = tot / reps;
    });
}

mlvs_status mlvs_step_stages(mlvs_ctx c, int* stages, int* count) {
    return guarded([&] {
        if (!c || !count) fail(MLVS_E_ARG, "null argument");
        const std::vector<int> st = step_stages(c);
        if (stages)
            for (size_t k = 0; k < st.size(); ++k) stages[k] = st[k];
        *count = (int)st.size();
    });
}

mlvs_status mlvs_stage_size(mlvs_ctx c, int stage, int64_t* items, double* points) {
    return guarded([&] {
        if (!c || stage < 0 || stage > 9) fail(MLVS_E_ARG, "bad arguments");
        int64_t ni = 0;
        double np = 0.0;
        switch (stage) {
        case 0: case 5: case 6: case 8: case 9:
            ni = c->mesh.n_cells;
            np = stage == 6 ? (double)c->mesh.n_cells * c->base.N : c->step_points;
            break;
        case 1: ni = c->n_ghosts; for (auto& L : c->levels) np += (double)L->n_ghost * L->N; break;
        case 2: case 3: case 7: {
            // same-level interior faces and boundary faces: each carries its level's points
            ni = c->n_faces + c->n_bfaces;
            for (auto& f : c->mesh.faces) {
                const int a = c->cell_level[f.L];
                if (a == c->cell_level[f.R]) np += c->levels[a]->N;
            }
            for (auto& f : c->mesh.bfaces) np += c->levels[c->cell_level[f.L]]->N;
            break;
        }
        case 4: ni = c->n_xfaces; np = c->step_iface_points; break;
        }
        if (items) *items = ni;
        if (points) *points = np;
    });
}

mlvs_status mlvs_memory(mlvs_ctx c, size_t* bytes) {
    return guarded([&] {
        if (!c || !bytes) fail(MLVS_E_ARG, "null argument");
        *bytes = c->dm.bytes;
    });
}

mlvs_status mlvs_positivity_counts(mlvs_ctx c, int64_t* applied, int64_t* failed) {
    return guarded([&] {
        if (!c || !applied || !failed) fail(MLVS_E_ARG, "null argument");
        unsigned long long v[3] = {0, 0, 0};
        hip_check(hipMemcpyAsync(v, c->d_neg, 24, hipMemcpyDeviceToHost, c->st), "D2H");
        sync(c);
        *applied = (int64_t)v[1];
        *failed = (int64_t)v[2];
    });
}

mlvs_status mlvs_neg_count(mlvs_ctx c, int64_t* count) {
    return guarded([&] {
        if (!c || !count) fail(MLVS_E_ARG, "null argument");
        unsigned long long v = 0;
        hip_check(hipMemcpyAsync(&v, c->d_neg, 8, hipMemcpyDeviceToHost, c->st), "D2H");
        sync(c);
        *count = (int64_t)v;
    });
}

mlvs_status mlvs_level_info(mlvs_ctx c, int* n_levels, int32_t* npts, int32_t* ncells, int64_t* n_cross) {
    return guarded([&] {
        if (!c || !n_levels) fail(MLVS_E_ARG, "null argument");
        *n_levels = (int)c->levels.size();
        for (size_t l = 0; l < c->levels.size(); ++l) {
            if (npts) npts[l] = c->levels[l]->N;
            if (ncells) ncells[l] = c->levels[l]->n_cells;
        }
        if (n_cross) *n_cross = c->n_cross;
    });
}

mlvs_status mlvs_level_kappa(mlvs_ctx c, int level, uint8_t* out) {
    return guarded([&] {
        if (!c || !out || level < 0 || level >= (int)c->levels.size()) fail(MLVS_E_ARG, "bad level");
        std::copy(c->levels[level]->kappa.begin(), c->levels[level]->kappa.end(), out);
    });
}

mlvs_status mlvs_cell_levels(mlvs_ctx c, int32_t* out) {
    return guarded([&] {
        if (!c || !out) fail(MLVS_E_ARG, "null argument");
        std::copy(c->cell_level.begin(), c->cell_level.end(), out);
    });
}

static void copy_cell(mlvs_ctx c, int64_t cell, double* g, double* h, const double* gi, const double* hi) {
    const Level& L = *c->levels[c->cell_level[cell]];
    const size_t off = (size_t)c->cell_slot[cell] * L.stride * c->elt();
    const size_t nb = (size_t)L.N * c->elt();
    std::vector<char> buf(nb);
    for (int comp = 0; comp < 2; ++comp) {
        char* base = static_cast<char*>(comp ? L.h : L.g) + off;
        double* o = comp ? h : g;
        const double* in = comp ? hi : gi;
        if (o) {
            hip_check(hipMemcpyAsync(buf.data(), base, nb, hipMemcpyDeviceToHost, c->st), "D2H");
            sync(c);
            for (int i = 0; i < L.N; ++i)
                o[L.canon_of[i]] = c->prec == 32 ? (double)reinterpret_cast<float*>(buf.data())[i]
                                                 : reinterpret_cast<double*>(buf.data())[i];
        }
        if (in) {
            for (int i = 0; i < L.N; ++i) {
                if (c->prec == 32) reinterpret_cast<float*>(buf.data())[i] = (float)in[L.canon_of[i]];
                else reinterpret_cast<double*>(buf.data())[i] = in[L.canon_of[i]];
            }
            hip_check(hipMemcpyAsync(base, buf.data(), nb, hipMemcpyHostToDevice, c->st), "H2D");
            sync(c);
        }
    }
}

mlvs_status mlvs_get_f(mlvs_ctx c, int64_t cell, double* g, double* h, int32_t* npts) {
    return guarded([&] {
        if (!c || cell < 0 || cell >= c->mesh.n_cells) fail(MLVS_E_ARG, "bad cell");
        if (npts) *npts = c->levels[c->cell_level[cell]]->N;
        if (g || h) copy_cell(c, cell, g, h, nullptr, nullptr);
    });
}

mlvs_status mlvs_set_f(mlvs_ctx c, int64_t cell, const double* g, const double* h) {
    return guarded([&] {
        if (!c || !g || !h || cell < 0 || cell >= c->mesh.n_cells) fail(MLVS_E_ARG, "bad arguments");
        copy_cell(c, cell, nullptr, nullptr, g, h);
        c->state_ready = true;
        c->mom_valid = false;
    c->prep_valid = false;
    });
}

static void bulk_state(mlvs_ctx c, double* g, double* h, const double* gi, const double* hi) {
    // per level: copy the whole state block once, then scatter in cell order
    std::vector<size_t> offset(c->mesh.n_cells);
    size_t tot = 0;
    for (int cc = 0; cc < c->mesh.n_cells; ++cc) {
        offset[cc] = tot;
        tot += c->levels[c->cell_level[cc]]->N;
    }
    for (size_t l = 0; l < c->levels.size(); ++l) {
        Level& L = *c->levels[l];
        const size_t nb = (size_t)L.n_cells * L.stride * c->elt();
        if (nb == 0) continue;
        std::vector<char> buf(nb, 0);
        for (int comp = 0; comp < 2; ++comp) {
            char* base = static_cast<char*>(comp ? L.h : L.g);
            const double* in = comp ? hi : gi;
            double* o = comp ? h : g;
            if (o) {
                hip_check(hipMemcpyAsync(buf.data(), base, nb, hipMemcpyDeviceToHost, c->st), "D2H");
                sync(c);
            }
            for (int cc = 0; cc < c->mesh.n_cells; ++cc) {
                if (c->cell_level[cc] != (int)l) continue;
                const size_t r = (size_t)c->cell_slot[cc] * L.stride;
                for (int i = 0; i < L.N; ++i) {
                    const size_t ci = offset[cc] + L.canon_of[i];
                    if (o) o[ci] = c->prec == 32 ? (double)reinterpret_cast<float*>(buf.data())[r + i]
                                                 : reinterpret_cast<double*>(buf.data())[r + i];
                    if (in) {
                        if (c->prec == 32) reinterpret_cast<float*>(buf.data())[r + i] = (float)in[ci];
                        else reinterpret_cast<double*>(buf.data())[r + i] = in[ci];
                    }
                }
            }
            if (in) {
                hip_check(hipMemcpyAsync(base, buf.data(), nb, hipMemcpyHostToDevice, c->st), "H2D");
                sync(c);
            }
        }
    }
}

mlvs_status mlvs_get_state(mlvs_ctx c, double* g, double* h) {
    return guarded([&] {
        if (!c || !g || !h) fail(MLVS_E_ARG, "null argument");
        bulk_state(c, g, h, nullptr, nullptr);
    });
}

mlvs_status mlvs_set_state(mlvs_ctx c, const double* g, const double* h) {
    return guarded([&] {
        if (!c || !g || !h) fail(MLVS_E_ARG, "null argument");
        bulk_state(c, nullptr, nullptr, g, h);
        c->state_ready = true;
        c->mom_valid = false;
    c->prep_valid = false;
    });
}

mlvs_status mlvs_set_levels(mlvs_ctx c, int n_levels, const uint8_t* kappa, const int32_t* cell_level) {
    return guarded([&] {
        if (!c || !kappa || !cell_level || n_levels < 1) fail(MLVS_E_ARG, "bad arguments");
        if (c->phys.dim != 2) fail(MLVS_E_STATE, "levels need dim = 2");
        if (!c->state_ready) fail(MLVS_E_STATE, "state not initialised");
        std::vector<std::unique_ptr<Level>> nl;
        for (int l = 0; l < n_levels; ++l) {
            check_kappa(c->base, kappa + (size_t)l * c->base.Nb);
            nl.push_back(build_level(c->base, std::vector<uint8_t>(kappa + (size_t)l * c->base.Nb,
                                                                    kappa + (size_t)(l + 1) * c->base.Nb)));
        }
        std::vector<int> cl(cell_level, cell_level + c->mesh.n_cells);
        for (int v : cl)
            if (v < 0 || v >= n_levels) fail(MLVS_E_ARG, "cell level out of range");
        install_levels(c, std::move(nl), cl);
    });
}

mlvs_status mlvs_adapt(mlvs_ctx c, mlvs_adapt_report* rep) {
    return guarded([&] {
        if (!c) fail(MLVS_E_ARG, "null context");
        if (!c->adaptive) fail(MLVS_E_STATE, "context was created without adaptation parameters");
        if (!c->state_ready) fail(MLVS_E_STATE, "state not initialised");
        if (rep) *rep = mlvs_adapt_report{};
        if (c->sel_K > 0 && c->sel_on) adapt_learned(c, rep);
        else adapt_now(c, rep);
    });
}

mlvs_status mlvs_criterion(mlvs_ctx c, uint8_t* out) {
    return guarded([&] {
        if (!c || !out) fail(MLVS_E_ARG, "null argument");
        if (!c->adaptive) fail(MLVS_E_STATE, "context was created without adaptation parameters");
        if (!c->state_ready) fail(MLVS_E_STATE, "state not initialised");
        run_criterion(c);
        hip_check(hipMemcpyAsync(out, c->d_kcell, (size_t)c->mesh.n_cells * c->base.Nb, hipMemcpyDeviceToHost, c->st),
                  "D2H");
        sync(c);
    });
}

}  // extern "C"

namespace {

void do_step(mlvs_ctx c) {
    const int n = c->mesh.n_cells;
    if (c->adaptive && c->ap.interval > 0 && c->step_count % c->ap.interval == 0) {
        if (mlvs_adapt(c, nullptr) != MLVS_OK) throw Fail{MLVS_E_STATE, g_last_error};
    }
    ensure_moments(c);
    if ((c->fused || c->persistent) && !c->prep_valid) {
        // the fused and persistent steps start from a prepared cell stage (the
        // previous step's update prepares the next one)
        hip_check(launch_stage(c, 0), "cell stage launch");
        c->prep_valid = true;
    }
    if (c->use_graph) {
        if (!c->gexec) {
            hip_check(hipStreamBeginCapture(c->st, hipStreamCaptureModeThreadLocal), "begin capture");
            hipError_t e = launch_step_kernels(c);
            hipGraph_t g = nullptr;
            hipError_t e2 = hipStreamEndCapture(c->st, &g);
            hip_check(e, "captured launch");
            hip_check(e2, "end capture");
            c->graph = g;
            hip_check(hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0), "graph instantiate");
            ++c->n_captures;
        }
        hip_check(hipGraphLaunch(c->gexec, c->st), "graph launch");
        ++c->n_graph_launches;
    } else {
        hip_check(launch_step_kernels(c), "step launch");
    }
    c->prep_valid = c->fused || c->persistent;
    ++c->step_count;
    c->cnt_updates += c->step_points;
    c->cnt_iface += c->step_iface_points;
}

// The stages one step launches, in order.
std::vector<int> step_stages(mlvs_ctx c) {
    if (c->persistent) return {9};
    if (c->fused) return {1, 7, 4, 8};
    return {0, 1, 2, 3, 4, 5};
}

hipError_t launch_step_kernels(mlvs_ctx c) {
    if (c->persistent) return launch_stage(c, 9);
    // cross-level faces (stage 4) beside the same-level face stages: both read
    // the cell stage's rows and the ghost rows, and they write distinct rows
    const bool fork = c->n_xfaces > 0 && c->side_st;
    for (int stage : step_stages(c)) {
        hipError_t e = hipSuccess;
        if (fork && stage == 4) continue;
        if (fork && (stage == 2 || stage == 7)) {
            if ((e = hipEventRecord(c->ev_fork, c->st)) != hipSuccess) return e;
            if ((e = hipStreamWaitEvent(c->side_st, c->ev_fork, 0)) != hipSuccess) return e;
            if ((e = launch_stage(c, 4, c->side_st)) != hipSuccess) return e;
            if ((e = hipEventRecord(c->ev_join, c->side_st)) != hipSuccess) return e;
        }
        if (fork && (stage == 5 || stage == 8))
            if ((e = hipStreamWaitEvent(c->st, c->ev_join, 0)) != hipSuccess) return e;
        if ((e = launch_stage(c, stage)) != hipSuccess) return e;
    }
    return hipSuccess;
}

// Stages of the step: 0 cell, 1 neighbour mapping (ghost rows), 2 face
// reconstruction and 3 face target (same-level and boundary faces), 4
// cross-level faces, 5 update; fused forms 7 (2 + 3) and 8 (5 + the next
// step's 0).  6 (criterion) is timed apart.
hipError_t launch_stage(mlvs_ctx c, int stage, hipStream_t on) {
    const int n = c->mesh.n_cells;
    const int nf = c->n_faces + c->n_bfaces;
    switch (stage) {
    case 0: return launch_cell_prep(c->prec, c->st, c->d_lv, c->d_cell_lev, c->d_cell_slot, c->d_order, n, c->ph,
                                    c->d_params, c->d_cmom, c->chunk, c->variant[0]);
    case 1: return launch_ghost(c->prec, c->st, c->d_lv, c->d_ghosts, c->n_ghosts, c->d_cell_lev, c->d_cell_slot,
                                c->d_params, c->ph, c->d_neg);
    case 2: return launch_face_rec(c->prec, c->st, c->d_lv, c->d_faces, nf, c->d_cell_slot, c->d_cell_nbr, c->d_geom,
                                   c->d_params, c->ph, c->d_fmom, c->chunk, c->nch, c->variant[2]);
    case 3: return launch_face_target(c->prec, c->st, c->d_lv, c->d_faces, nf, c->d_bcs, c->ph, c->d_fmom,
                                      c->d_fpar, c->chunk, c->variant[3]);
    case 4: return launch_xface(c->prec, on ? on : c->st, c->d_lv, c->d_xfaces, c->n_xfaces, c->d_cell_slot, c->d_cell_nbr,
                                c->d_geom, c->d_params, c->ph, c->d_neg, c->variant[4]);
    case 5: return launch_update(c->prec, c->st, c->d_lv, c->d_cell_lev, c->d_cell_slot, c->d_order, n, c->d_geom,
                                 c->d_cell_frow, c->d_faces, c->d_fpar, c->d_params, c->ph, c->d_cmom, c->chunk,
                                 c->nch, c->variant[5]);
    case 7: return launch_face_full(c->prec, c->st, c->d_lv, c->d_faces, nf, c->d_cell_slot, c->d_cell_nbr,
                                    c->d_geom, c->d_params, c->d_bcs, c->ph, c->d_fpar, c->variant[7]);
    case 9: return launch_step_persistent(c->prec, c->st, c->d_args, c->d_sync, c->ph, c->variant[9],
                                          &c->persistent_grid);
    case 8: return launch_update_cell(c->prec, c->st, c->d_lv, c->d_cell_lev, c->d_cell_slot, c->d_order, n,
                                      c->d_geom, c->d_cell_frow, c->d_faces, c->d_fpar, c->d_params, c->ph,
                                      c->d_cmom, c->variant[8]);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace
