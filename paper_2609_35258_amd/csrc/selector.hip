// Learned level selector for gfx950: per-cell features, a 10 -> 64 -> 64 -> K
// ReLU network trained with softmax cross-entropy and Adam in FP32, BF16
// inference, and the tail-mass check that sends doubtful predictions back to
// the distribution-function criterion.
//
// Parameter layout (float): W1 [64][10], b1 [64], W2 [64][64], b2 [64],
// W3 [K][64], b3 [K], mean [10], std [10].
#include "mlvs_impl.h"

#include <cmath>
#include <mutex>

namespace mlvs {

constexpr int NF = 10;
constexpr int NH = 64;
constexpr int KMAX = 16;

__host__ __device__ inline int mlp_offsets(int K, int which) {
    const int o[9] = {0,
                      NH * NF,
                      NH * NF + NH,
                      NH * NF + NH + NH * NH,
                      NH * NF + NH + NH * NH + NH,
                      NH * NF + NH + NH * NH + NH + K * NH,
                      NH * NF + NH + NH * NH + NH + K * NH + K,
                      NH * NF + NH + NH * NH + NH + K * NH + K + NF,
                      NH * NF + NH + NH * NH + NH + K * NH + K + 2 * NF};
    return o[which];
}

int mlp_nparams(int K) { return mlp_offsets(K, 8); }

// ---------------------------------------------------------------------------
// features: per cell from its (rho, u, v, T, qx, qy, sxx, sxy) and neighbours
// ---------------------------------------------------------------------------
__global__ void k_features(const double* __restrict__ f8, const int* __restrict__ nbr_cell,
                           const CellGeom* __restrict__ geom, int n_cells, double R, double T_ref,
                           double mu_ref, double omega, int unstructured, float* __restrict__ out) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cells) return;
    const double* m = f8 + 8 * (size_t)c;
    const double rho = m[0], u = m[1], v = m[2], T = m[3];
    const double p = rho * R * T, cs = sqrt(R * T);
    // gradient of rho: central difference per index direction (one-sided at a
    // boundary, zero without neighbours), mapped through [t_i; t_j]^-1
    const CellGeom g = geom[c];
    double sdir[2];
    for (int d = 0; d < 2; ++d) {
        const int lo = nbr_cell[4 * c + 2 * d], hi = nbr_cell[4 * c + 2 * d + 1];
        if (lo >= 0 && hi >= 0) sdir[d] = (f8[8 * (size_t)hi] - f8[8 * (size_t)lo]) / (g.dist[2 * d] + g.dist[2 * d + 1]);
        else if (hi >= 0) sdir[d] = (f8[8 * (size_t)hi] - rho) / g.dist[2 * d + 1];
        else if (lo >= 0) sdir[d] = (rho - f8[8 * (size_t)lo]) / g.dist[2 * d];
        else sdir[d] = 0.0;
    }
    double gx = g.G[0] * sdir[0] + g.G[1] * sdir[1];
    double gy = g.G[2] * sdir[0] + g.G[3] * sdir[1];
    if (unstructured) {
        // least squares over the face neighbours (slot k: the k-th edge); a
        // boundary ghost carries no difference
        gx = 0.0;
        gy = 0.0;
        for (int k = 0; k < 4; ++k) {
            const int nb = nbr_cell[4 * c + k];
            if (nb < 0) continue;
            const double d = f8[8 * (size_t)nb] - rho;
            gx += g.lx[k] * d;
            gy += g.ly[k] * d;
        }
    }
    const double grad = sqrt(gx * gx + gy * gy);
    const double mu = mu_ref * pow(T / T_ref, omega);
    const double lam = (mu / p) * sqrt(M_PI * R * T / 2.0);
    const double dx = sqrt(g.vol);
    float* o = out + (size_t)NF * c;
    o[0] = (float)log(rho);
    o[1] = (float)(u / sqrt(R * T_ref));
    o[2] = (float)(v / sqrt(R * T_ref));
    o[3] = (float)log(T / T_ref);
    o[4] = (float)(m[4] / (p * cs));
    o[5] = (float)(m[5] / (p * cs));
    o[6] = (float)(m[6] / p);
    o[7] = (float)(m[7] / p);
    o[8] = (float)log1p(dx * grad / rho);
    o[9] = (float)log10(lam / dx);
}

// ---------------------------------------------------------------------------
// network: forward + per-sample deltas (thread per sample), weight gradients
// (thread per weight, fixed-order sum over the batch), Adam
// ---------------------------------------------------------------------------
__device__ __forceinline__ float to_bf16(float x) {
    // round to nearest even on the upper 16 bits
    unsigned int u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return x;
    u += 0x7fffu + ((u >> 16) & 1u);
    return __uint_as_float(u & 0xffff0000u);
}

template <bool BF16>
__device__ __forceinline__ void mlp_fwd_one(const float* __restrict__ P, int K, const float* x, float* z1, float* a1,
                                            float* z2, float* a2, float* z3) {
    const float* W1 = P;
    const float* b1 = P + mlp_offsets(K, 1);
    const float* W2 = P + mlp_offsets(K, 2);
    const float* b2 = P + mlp_offsets(K, 3);
    const float* W3 = P + mlp_offsets(K, 4);
    const float* b3 = P + mlp_offsets(K, 5);
    const float* mu = P + mlp_offsets(K, 6);
    const float* sd = P + mlp_offsets(K, 7);
    float xn[NF];
    for (int k = 0; k < NF; ++k) {
        xn[k] = (x[k] - mu[k]) / sd[k];
        if (BF16) xn[k] = to_bf16(xn[k]);
    }
    for (int j = 0; j < NH; ++j) {
        float s = b1[j];
        for (int k = 0; k < NF; ++k) s += (BF16 ? to_bf16(W1[j * NF + k]) : W1[j * NF + k]) * xn[k];
        z1[j] = s;
        a1[j] = s > 0.f ? s : 0.f;
        if (BF16) a1[j] = to_bf16(a1[j]);
    }
    for (int j = 0; j < NH; ++j) {
        float s = b2[j];
        for (int k = 0; k < NH; ++k) s += (BF16 ? to_bf16(W2[j * NH + k]) : W2[j * NH + k]) * a1[k];
        z2[j] = s;
        a2[j] = s > 0.f ? s : 0.f;
        if (BF16) a2[j] = to_bf16(a2[j]);
    }
    for (int j = 0; j < K; ++j) {
        float s = b3[j];
        for (int k = 0; k < NH; ++k) s += (BF16 ? to_bf16(W3[j * NH + k]) : W3[j * NH + k]) * a2[k];
        z3[j] = s;
    }
}

// Forward and backward deltas of one batch.  Stores normalised inputs,
// activations and the deltas dz1, dz2, dz3 per sample, the probabilities and
// the per-sample loss (for a fixed-order sum afterwards).
__global__ void k_mlp_fwd_bwd(const float* __restrict__ P, int K, const float* __restrict__ X,
                              const int* __restrict__ y, const int* __restrict__ idx, int B, float* __restrict__ XN,
                              float* __restrict__ A1, float* __restrict__ A2, float* __restrict__ D1,
                              float* __restrict__ D2, float* __restrict__ D3, float* __restrict__ prob,
                              float* __restrict__ lossv) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const int s = idx ? idx[b] : b;
    float x[NF], z1[NH], a1[NH], z2[NH], a2[NH], z3[KMAX];
    for (int k = 0; k < NF; ++k) x[k] = X[(size_t)s * NF + k];
    mlp_fwd_one<false>(P, K, x, z1, a1, z2, a2, z3);
    const float* mu = P + mlp_offsets(K, 6);
    const float* sd = P + mlp_offsets(K, 7);
    for (int k = 0; k < NF; ++k) XN[(size_t)b * NF + k] = (x[k] - mu[k]) / sd[k];
    float zmax = z3[0];
    for (int j = 1; j < K; ++j) zmax = fmaxf(zmax, z3[j]);
    float e[KMAX], se = 0.f;
    for (int j = 0; j < K; ++j) { e[j] = expf(z3[j] - zmax); se += e[j]; }
    const int yy = y[s];
    float d3[KMAX];
    for (int j = 0; j < K; ++j) {
        const float pj = e[j] / se;
        if (prob) prob[(size_t)b * K + j] = pj;
        d3[j] = (pj - (j == yy ? 1.f : 0.f)) / (float)B;
        D3[(size_t)b * K + j] = d3[j];
    }
    lossv[b] = -(z3[yy] - zmax - logf(se));
    const float* W2 = P + mlp_offsets(K, 2);
    const float* W3 = P + mlp_offsets(K, 4);
    float d2[NH];
    for (int k = 0; k < NH; ++k) {
        float s2 = 0.f;
        for (int j = 0; j < K; ++j) s2 += d3[j] * W3[j * NH + k];
        d2[k] = z2[k] > 0.f ? s2 : 0.f;
        D2[(size_t)b * NH + k] = d2[k];
        A2[(size_t)b * NH + k] = a2[k];
    }
    for (int k = 0; k < NH; ++k) {
        float s1 = 0.f;
        for (int j = 0; j < NH; ++j) s1 += d2[j] * W2[j * NH + k];
        D1[(size_t)b * NH + k] = z1[k] > 0.f ? s1 : 0.f;
        A1[(size_t)b * NH + k] = a1[k];
    }
}

// Gradient of every trainable parameter: sum over the batch in sample order.
__global__ void k_mlp_grad(int K, int B, const float* __restrict__ XN, const float* __restrict__ A1,
                           const float* __restrict__ A2, const float* __restrict__ D1, const float* __restrict__ D2,
                           const float* __restrict__ D3, float* __restrict__ G) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int ntr = mlp_offsets(K, 6);
    if (t >= ntr) return;
    const float *D, *A;
    int nd, na, i, j = -1;
    if (t < mlp_offsets(K, 1)) { D = D1; A = XN; nd = NH; na = NF; i = t / NF; j = t % NF; }
    else if (t < mlp_offsets(K, 2)) { D = D1; A = nullptr; nd = NH; na = 0; i = t - mlp_offsets(K, 1); }
    else if (t < mlp_offsets(K, 3)) { D = D2; A = A1; nd = NH; na = NH; i = (t - mlp_offsets(K, 2)) / NH; j = (t - mlp_offsets(K, 2)) % NH; }
    else if (t < mlp_offsets(K, 4)) { D = D2; A = nullptr; nd = NH; na = 0; i = t - mlp_offsets(K, 3); }
    else if (t < mlp_offsets(K, 5)) { D = D3; A = A2; nd = K; na = NH; i = (t - mlp_offsets(K, 4)) / NH; j = (t - mlp_offsets(K, 4)) % NH; }
    else { D = D3; A = nullptr; nd = K; na = 0; i = t - mlp_offsets(K, 5); }
    float s = 0.f;
    for (int b = 0; b < B; ++b) s += D[(size_t)b * nd + i] * (A ? A[(size_t)b * na + j] : 1.f);
    G[t] = s;
}

__global__ void k_adam(float* __restrict__ P, const float* __restrict__ G, float* __restrict__ M,
                       float* __restrict__ V, int n, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const float g = G[t];
    const float m = b1 * M[t] + (1.f - b1) * g;
    const float v = b2 * V[t] + (1.f - b2) * g * g;
    M[t] = m;
    V[t] = v;
    P[t] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
}

// Single-wave fixed-order sum of n floats (loss) into double.
__global__ void k_sumf(const float* __restrict__ x, int n, double* __restrict__ out) {
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 64) s += (double)x[i];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (threadIdx.x == 0) *out = s;
}

// Inference (FP32 or BF16-rounded weights and activations, FP32 accumulation).
template <bool BF16>
__global__ void k_mlp_predict(const float* __restrict__ P, int K, const float* __restrict__ X, int B,
                              int* __restrict__ cls, float* __restrict__ prob) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    float x[NF], z1[NH], a1[NH], z2[NH], a2[NH], z3[KMAX];
    for (int k = 0; k < NF; ++k) x[k] = X[(size_t)b * NF + k];
    mlp_fwd_one<BF16>(P, K, x, z1, a1, z2, a2, z3);
    int best = 0;
    float zmax = z3[0];
    for (int j = 1; j < K; ++j)
        if (z3[j] > zmax) { zmax = z3[j]; best = j; }
    cls[b] = best;
    if (prob) {
        float se = 0.f;
        for (int j = 0; j < K; ++j) se += expf(z3[j] - zmax);
        for (int j = 0; j < K; ++j) prob[(size_t)b * K + j] = expf(z3[j] - zmax) / se;
    }
}

// ---------------------------------------------------------------------------
// tail-mass check: reject a predicted level if any block it merges carries an
// indicator I_B = max(sum M1, sum M2) above C_split on the cell's distribution
// ---------------------------------------------------------------------------
template <typename S>
__global__ __launch_bounds__(256) void k_tail_check(const LevelDesc* __restrict__ lvs,
                                                    const int* __restrict__ cell_lev,
                                                    const int* __restrict__ cell_slot, int n_cells,
                                                    const int* __restrict__ ptb_all, const int* __restrict__ ptb_off,
                                                    const uint8_t* __restrict__ kappa_all,
                                                    const int* __restrict__ pred, const double* __restrict__ bw,
                                                    int nx, int ny, double C_split, int* __restrict__ accept) {
    const int lane = threadIdx.x & 63;
    const int c = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + (threadIdx.x >> 6)));
    if (c >= n_cells) return;
    const int lev = cell_lev[c];
    const LevelDesc& L = lvs[lev];
    const size_t row = (size_t)cell_slot[c] * L.stride;
    const S* g = reinterpret_cast<const S*>(L.g) + row;
    const S* h = reinterpret_cast<const S*>(L.h) + row;
    const int* ptb = ptb_all + ptb_off[lev];
    const int nbx = nx / 2, nby = ny / 2, Nb = nbx * nby;
    const uint8_t* kp = kappa_all + (size_t)pred[c] * Nb;
    double t[2] = {0.0, 0.0};
    for (int b = lane; b < nx * ny; b += 64) {
        const int p = ptb[b];
        const double gp = (double)g[p];
        const double xp = L.xi_x[p], yp = L.xi_y[p];
        t[0] += bw[b] * gp;
        t[1] += 0.5 * bw[b] * ((double)h[p] + (xp * xp + yp * yp) * gp);
    }
    for (int k = 0; k < 2; ++k)
        for (int off = 32; off > 0; off >>= 1) t[k] += __shfl_xor(t[k], off, 64);
    int bad = 0;
    for (int bb = lane; bb < Nb; bb += 64) {
        const int s = kp[bb];
        if (s == 0) continue;
        const int bx = bb % nbx, by = bb / nbx;
        const int csz = 1 << (s - 1);
        if ((bx % csz) != 0 || (by % csz) != 0) continue;       // anchor of its merged block only
        const int size = 1 << s, X0 = (bx / csz) * size, Y0 = (by / csz) * size;
        double m1 = 0.0, m2 = 0.0;
        for (int iy = Y0; iy < Y0 + size; ++iy)
            for (int ix = X0; ix < X0 + size; ++ix) {
                const int b = ix + nx * iy, p = ptb[b];
                const double gp = (double)g[p];
                const double xp = L.xi_x[p], yp = L.xi_y[p];
                m1 += bw[b] * gp;
                m2 += 0.5 * bw[b] * ((double)h[p] + (xp * xp + yp * yp) * gp);
            }
        if (fmax(m1 / t[0], m2 / t[1]) > C_split) bad = 1;
    }
    bad = __any(bad);
    if (lane == 0) accept[c] = bad ? 0 : 1;
}

// Label rule on the device: fewest-point catalogue level whose enclosing mask
// is no coarser than the cell's criterion mask anywhere (-1 if none).
__global__ void k_labels(const uint8_t* __restrict__ kcell, int n_cells, int Nb, const uint8_t* __restrict__ kappa_all,
                         const int* __restrict__ order, int K, int* __restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int c = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + (threadIdx.x >> 6)));
    if (c >= n_cells) return;
    const uint8_t* kc = kcell + (size_t)c * Nb;
    int found = -1;
    for (int q = 0; q < K && found < 0; ++q) {
        const int l = order[q];
        const uint8_t* kl = kappa_all + (size_t)l * Nb;
        int bad = 0;
        for (int b = lane; b < Nb; b += 64) bad |= kl[b] > kc[b];
        if (!__any(bad)) found = l;
    }
    if (lane == 0) out[c] = found;
}

// ---------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------
hipError_t launch_features(hipStream_t st, const double* f8, const int* nbr_cell, const CellGeom* geom, int n,
                           double R, double T_ref, double mu_ref, double omega, int unstructured, float* out) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_features, dim3((n + 255) / 256), dim3(256), 0, st, f8, nbr_cell, geom, n, R, T_ref, mu_ref,
                       omega, unstructured, out);
    return hipGetLastError();
}

hipError_t launch_mlp_fwd_bwd(hipStream_t st, const float* P, int K, const float* X, const int* y, const int* idx,
                              int B, float* XN, float* A1, float* A2, float* D1, float* D2, float* D3, float* prob,
                              float* lossv, double* loss_sum) {
    hipLaunchKernelGGL(k_mlp_fwd_bwd, dim3((B + 127) / 128), dim3(128), 0, st, P, K, X, y, idx, B, XN, A1, A2, D1, D2,
                       D3, prob, lossv);
    hipLaunchKernelGGL(k_sumf, dim3(1), dim3(64), 0, st, lossv, B, loss_sum);
    return hipGetLastError();
}

hipError_t launch_mlp_grad(hipStream_t st, int K, int B, const float* XN, const float* A1, const float* A2,
                           const float* D1, const float* D2, const float* D3, float* G) {
    const int n = mlp_offsets(K, 6);
    hipLaunchKernelGGL(k_mlp_grad, dim3((n + 255) / 256), dim3(256), 0, st, K, B, XN, A1, A2, D1, D2, D3, G);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// forward/backward without device allocation: the intermediate values live in
// a fixed device array of the library
// ---------------------------------------------------------------------------
// Layout (bytes): [0, 256) the loss sum when the caller wants none; then, for
// at most NOALLOC_MAX_BATCH samples, XN [B][10], A1, A2, D1, D2 [B][64],
// D3 [B][16], per-sample losses [B] (floats).  Each GPU holds its own copy
// until the process ends; calls on one GPU share it.
constexpr size_t NOALLOC_FLOATS_PER_SAMPLE = NF + 4 * NH + KMAX + 1;
constexpr size_t NOALLOC_BYTES = 256 + sizeof(float) * NOALLOC_FLOATS_PER_SAMPLE * NOALLOC_MAX_BATCH;
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

// Zero the gradient entries the gradient kernel does not write (the
// standardisation block): a fill kernel, so the launch sequence holds no
// memset node when a caller captures it in a graph.
__global__ void k_fill_zero(float* __restrict__ p, int n) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = 0.f;
}

// The array's device address, looked up once per device (with that device
// current) and kept: in host code the array's name is not a device address.
static hipError_t scratch_address(unsigned char** out) {
    constexpr int MAXDEV = 64;
    static unsigned char* addr[MAXDEV] = {};
    static std::mutex m;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAXDEV) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(m);
    if (!addr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = static_cast<unsigned char*>(ptr);
    }
    *out = addr[dev];
    return hipSuccess;
}

size_t noalloc_scratch_bytes() { return NOALLOC_BYTES; }

hipError_t launch_mlp_eval_noalloc(hipStream_t st, const float* P, int K, const float* X, const int* y, int B,
                                   float* prob, float* grad, double* loss_sum) {
    if (B < 1 || B > NOALLOC_MAX_BATCH || K < 2 || K > KMAX) return hipErrorInvalidValue;
    unsigned char* base = nullptr;
    hipError_t e = scratch_address(&base);
    if (e != hipSuccess) return e;
    double* ls = loss_sum ? loss_sum : reinterpret_cast<double*>(base);
    float* f = reinterpret_cast<float*>(base + 256);
    const size_t Bs = (size_t)B;
    float* XN = f;
    float* A1 = XN + NF * Bs;
    float* A2 = A1 + NH * Bs;
    float* D1 = A2 + NH * Bs;
    float* D2 = D1 + NH * Bs;
    float* D3 = D2 + NH * Bs;
    float* LV = D3 + KMAX * Bs;
    e = launch_mlp_fwd_bwd(st, P, K, X, y, nullptr, B, XN, A1, A2, D1, D2, D3, prob, LV, ls);
    if (e != hipSuccess || !grad) return e;
    const int ntr = mlp_offsets(K, 6), np = mlp_nparams(K);
    hipLaunchKernelGGL(k_fill_zero, dim3(1), dim3(64), 0, st, grad + ntr, np - ntr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return launch_mlp_grad(st, K, B, XN, A1, A2, D1, D2, D3, grad);
}

hipError_t launch_adam(hipStream_t st, float* P, const float* G, float* M, float* V, int n, float lr, float b1,
                       float b2, float eps, int t) {
    const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, st, P, G, M, V, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_mlp_predict(hipStream_t st, const float* P, int K, const float* X, int B, int bf16, int* cls,
                              float* prob) {
    if (B <= 0) return hipSuccess;
    if (bf16) hipLaunchKernelGGL(k_mlp_predict<true>, dim3((B + 127) / 128), dim3(128), 0, st, P, K, X, B, cls, prob);
    else hipLaunchKernelGGL(k_mlp_predict<false>, dim3((B + 127) / 128), dim3(128), 0, st, P, K, X, B, cls, prob);
    return hipGetLastError();
}

hipError_t launch_tail_check(int prec, hipStream_t st, const LevelDesc* lv, const int* cell_lev, const int* cell_slot,
                             int n, const int* ptb_all, const int* ptb_off, const uint8_t* kappa_all, const int* pred,
                             const double* bw, int nx, int ny, double C_split, int* accept) {
    if (n <= 0) return hipSuccess;
    if (prec == 32)
        hipLaunchKernelGGL(k_tail_check<float>, dim3((n + 3) / 4), dim3(256), 0, st, lv, cell_lev, cell_slot, n,
                           ptb_all, ptb_off, kappa_all, pred, bw, nx, ny, C_split, accept);
    else
        hipLaunchKernelGGL(k_tail_check<double>, dim3((n + 3) / 4), dim3(256), 0, st, lv, cell_lev, cell_slot, n,
                           ptb_all, ptb_off, kappa_all, pred, bw, nx, ny, C_split, accept);
    return hipGetLastError();
}

hipError_t launch_labels(hipStream_t st, const uint8_t* kcell, int n, int Nb, const uint8_t* kappa_all,
                         const int* order, int K, int* out) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_labels, dim3((n + 3) / 4), dim3(256), 0, st, kcell, n, Nb, kappa_all, order, K, out);
    return hipGetLastError();
}

}  // namespace mlvs
