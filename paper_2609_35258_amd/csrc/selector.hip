// Learned level selector for gfx950: per-cell features, a 10 -> 64 -> 64 -> K
// ReLU network trained with softmax cross-entropy and Adam in FP32, BF16
// inference, and the tail-mass check that sends doubtful predictions back to
// the distribution-function criterion.
//
// Parameter layout (float): W1 [64][10], b1 [64], W2 [64][64], b2 [64],
// W3 [K][64], b3 [K], mean [10], std [10].
#include "mlvs_impl.h"

#include <algorithm>
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
// network, training and FP32 evaluation.  A workgroup of four waves takes 16
// samples at a time, four per wave; a wave's 64 lanes are the 64 hidden units,
// so each layer is a dot product per lane whose other operand is broadcast
// from LDS.  W2 and W3 are staged in LDS with a row pitch of 65 floats: a row
// per lane (forward) and a column per lane (backward) are both read without
// bank conflicts.  Training adds the backward pass and per-lane gradient
// accumulators; each workgroup writes one partial gradient, summed in a fixed
// order (waves, then workgroups), so results do not depend on timing.
// ---------------------------------------------------------------------------
constexpr int MW = 4;                              // waves per workgroup
constexpr int SPW = 4;                             // samples a wave carries together
constexpr int CHUNK = MW * SPW;                    // samples per workgroup pass
constexpr int WP = NH + 1;                         // LDS row pitch of W2 and W3
constexpr int NTR_MAX = NH * NF + NH + NH * NH + NH + KMAX * NH + KMAX;
constexpr int MAX_PART = 256;                      // partial gradients per batch

static int mlp_groups(int B) {
    const int ch = (B + CHUNK - 1) / CHUNK;
    return ch < MAX_PART ? ch : MAX_PART;
}

// LDS written by some lanes of a wave and then read by others of the same wave
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ float4 lds4(const float* p) { return *reinterpret_cast<const float4*>(p); }

// TRAIN: forward, backward and partial gradients (part [gridDim.x][ntr],
// lpart [gridDim.x] = sum of the per-sample losses); prob [B][K] optional.
// Otherwise forward only: cls [B] (first maximum) and prob [B][K] optional.
template <bool TRAIN>
__global__ __launch_bounds__(256) void k_mlp_batch(const float* __restrict__ P, int K, const float* __restrict__ X,
                                                   const int* __restrict__ y, const int* __restrict__ idx, int B,
                                                   float* __restrict__ prob, int* __restrict__ cls,
                                                   float* __restrict__ part, double* __restrict__ lpart) {
    __shared__ float sW2[NH * WP];
    __shared__ float sW3[KMAX * WP];
    __shared__ __align__(16) float sA1[MW][SPW][NH];
    __shared__ __align__(16) float sA2[MW][SPW][NH];
    __shared__ __align__(16) float sD2[MW][SPW][TRAIN ? NH : 4];
    __shared__ __align__(16) float sD3[MW][SPW][KMAX];
    __shared__ float sRed[TRAIN ? NTR_MAX : 1];
    __shared__ double sLoss[MW];
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    const float* W1 = P;
    const float* b1 = P + mlp_offsets(K, 1);
    const float* W2 = P + mlp_offsets(K, 2);
    const float* b2 = P + mlp_offsets(K, 3);
    const float* W3 = P + mlp_offsets(K, 4);
    const float* b3 = P + mlp_offsets(K, 5);
    const float* mu = P + mlp_offsets(K, 6);
    const float* sd = P + mlp_offsets(K, 7);
    for (int t = tid; t < NH * NH; t += 256) sW2[(t >> 6) * WP + (t & 63)] = W2[t];
    for (int t = tid; t < KMAX * NH; t += 256) sW3[(t >> 6) * WP + (t & 63)] = t < K * NH ? W3[t] : 0.f;
    float w1[NF];
    for (int k = 0; k < NF; ++k) w1[k] = W1[l * NF + k];
    const float bb1 = b1[l], bb2 = b2[l];
    // output layer: lane = (class j3, quarter q3 of the 64 inputs)
    const int j3 = l & 15, q3 = l >> 4;
    const bool cv = j3 < K;
    const float bb3 = cv ? b3[j3] : 0.f;
    __syncthreads();

    float g1[NF], g2[NH], g3[KMAX];
    for (int k = 0; k < NF; ++k) g1[k] = 0.f;
    for (int k = 0; k < NH; ++k) g2[k] = 0.f;
    for (int k = 0; k < KMAX; ++k) g3[k] = 0.f;
    float gb1 = 0.f, gb2 = 0.f, gb3 = 0.f;
    double wl = 0.0;
    const int nch = (B + CHUNK - 1) / CHUNK;
    for (int c = blockIdx.x; c < nch; c += gridDim.x) {
        int bpos[SPW], yy[SPW];
        bool ok[SPW];
        float xn[SPW][NF], a1[SPW], a2[SPW], z3[SPW], d3[SPW];
        for (int i = 0; i < SPW; ++i) {
            bpos[i] = c * CHUNK + w * SPW + i;
            ok[i] = bpos[i] < B;
            const int s = ok[i] ? (idx ? idx[bpos[i]] : bpos[i]) : 0;
            for (int k = 0; k < NF; ++k) xn[i][k] = ok[i] ? (X[(size_t)s * NF + k] - mu[k]) / sd[k] : 0.f;
            yy[i] = (TRAIN && ok[i]) ? y[s] : 0;
        }
        // first hidden layer (lane = unit)
        for (int i = 0; i < SPW; ++i) {
            float z = bb1;
            for (int k = 0; k < NF; ++k) z = fmaf(w1[k], xn[i][k], z);
            a1[i] = fmaxf(z, 0.f);
            sA1[w][i][l] = a1[i];
        }
        wave_sync();
        // second hidden layer: row l of W2 against the broadcast first layer
        {
            float z[SPW];
            for (int i = 0; i < SPW; ++i) z[i] = bb2;
            for (int k = 0; k < NH; k += 4) {
                const float* wr = sW2 + l * WP + k;
                const float w0 = wr[0], w1_ = wr[1], w2_ = wr[2], w3_ = wr[3];
                for (int i = 0; i < SPW; ++i) {
                    const float4 a = lds4(&sA1[w][i][k]);
                    z[i] = fmaf(w0, a.x, z[i]);
                    z[i] = fmaf(w1_, a.y, z[i]);
                    z[i] = fmaf(w2_, a.z, z[i]);
                    z[i] = fmaf(w3_, a.w, z[i]);
                }
            }
            for (int i = 0; i < SPW; ++i) {
                a2[i] = fmaxf(z[i], 0.f);
                sA2[w][i][l] = a2[i];
            }
        }
        wave_sync();
        // output layer: each quarter sums 16 inputs, two exchanges join them
        for (int i = 0; i < SPW; ++i) {
            float p = 0.f;
            for (int kk = 0; kk < 16; kk += 4) {
                const int k = q3 * 16 + kk;
                const float4 a = lds4(&sA2[w][i][k]);
                const float* wr = sW3 + j3 * WP + k;
                p = fmaf(wr[0], a.x, p);
                p = fmaf(wr[1], a.y, p);
                p = fmaf(wr[2], a.z, p);
                p = fmaf(wr[3], a.w, p);
            }
            p += __shfl_xor(p, 16, 64);
            p += __shfl_xor(p, 32, 64);
            z3[i] = p + bb3;
        }
        // softmax over the K classes (every quarter holds all of them)
        for (int i = 0; i < SPW; ++i) {
            float m = cv ? z3[i] : -INFINITY;
            for (int off = 8; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
            const float e = cv ? expf(z3[i] - m) : 0.f;
            float se = e;
            for (int off = 8; off > 0; off >>= 1) se += __shfl_xor(se, off, 64);
            const float pj = e / se;
            if (prob && ok[i] && q3 == 0 && cv) prob[(size_t)bpos[i] * K + j3] = pj;
            if (!TRAIN) {
                const unsigned long long at = __ballot(q3 == 0 && cv && z3[i] == m);
                if (ok[i] && l == 0) cls[bpos[i]] = at ? __ffsll(at) - 1 : 0;
            } else {
                d3[i] = ok[i] ? (pj - (j3 == yy[i] ? 1.f : 0.f)) / (float)B : 0.f;
                if (q3 == 0) sD3[w][i][j3] = d3[i];
                const float lz = z3[i] - m - logf(se);
                const float ly = __shfl(lz, yy[i], 64);
                if (ok[i]) wl -= (double)ly;
            }
        }
        if (TRAIN) {
            wave_sync();
            // back to the second hidden layer (lane = unit; classes >= K carry 0)
            float d2[SPW], d1[SPW];
            for (int i = 0; i < SPW; ++i) {
                float s = 0.f;
                for (int j = 0; j < KMAX; j += 4) {
                    const float4 d = lds4(&sD3[w][i][j]);
                    s = fmaf(d.x, sW3[(j + 0) * WP + l], s);
                    s = fmaf(d.y, sW3[(j + 1) * WP + l], s);
                    s = fmaf(d.z, sW3[(j + 2) * WP + l], s);
                    s = fmaf(d.w, sW3[(j + 3) * WP + l], s);
                }
                d2[i] = a2[i] > 0.f ? s : 0.f;
                sD2[w][i][l] = d2[i];
            }
            wave_sync();
            // back to the first hidden layer: column l of W2
            {
                float s[SPW];
                for (int i = 0; i < SPW; ++i) s[i] = 0.f;
                for (int j = 0; j < NH; j += 4) {
                    const float w0 = sW2[(j + 0) * WP + l], w1_ = sW2[(j + 1) * WP + l];
                    const float w2_ = sW2[(j + 2) * WP + l], w3_ = sW2[(j + 3) * WP + l];
                    for (int i = 0; i < SPW; ++i) {
                        const float4 d = lds4(&sD2[w][i][j]);
                        s[i] = fmaf(d.x, w0, s[i]);
                        s[i] = fmaf(d.y, w1_, s[i]);
                        s[i] = fmaf(d.z, w2_, s[i]);
                        s[i] = fmaf(d.w, w3_, s[i]);
                    }
                }
                for (int i = 0; i < SPW; ++i) d1[i] = a1[i] > 0.f ? s[i] : 0.f;
            }
            // gradient accumulators, samples in order: lane l owns W1 row l,
            // column l of W2 and W3, and bias entry l of each layer
            for (int i = 0; i < SPW; ++i) {
                for (int k = 0; k < NF; ++k) g1[k] = fmaf(d1[i], xn[i][k], g1[k]);
                gb1 += d1[i];
                gb2 += d2[i];
                for (int j = 0; j < NH; j += 4) {
                    const float4 d = lds4(&sD2[w][i][j]);
                    g2[j + 0] = fmaf(d.x, a1[i], g2[j + 0]);
                    g2[j + 1] = fmaf(d.y, a1[i], g2[j + 1]);
                    g2[j + 2] = fmaf(d.z, a1[i], g2[j + 2]);
                    g2[j + 3] = fmaf(d.w, a1[i], g2[j + 3]);
                }
                for (int j = 0; j < KMAX; j += 4) {
                    const float4 d = lds4(&sD3[w][i][j]);
                    g3[j + 0] = fmaf(d.x, a2[i], g3[j + 0]);
                    g3[j + 1] = fmaf(d.y, a2[i], g3[j + 1]);
                    g3[j + 2] = fmaf(d.z, a2[i], g3[j + 2]);
                    g3[j + 3] = fmaf(d.w, a2[i], g3[j + 3]);
                }
                gb3 += d3[i];
            }
        }
        wave_sync();
    }
    if (!TRAIN) return;
    // the workgroup's partial: waves added in order through LDS, the last
    // wave writes the sum
    const int o1 = mlp_offsets(K, 1), o2 = mlp_offsets(K, 2), o3 = mlp_offsets(K, 3);
    const int o4 = mlp_offsets(K, 4), o5 = mlp_offsets(K, 5), ntr = mlp_offsets(K, 6);
    float* out = part + (size_t)blockIdx.x * ntr;
    for (int r = 0; r < MW; ++r) {
        if (w == r) {
            auto put = [&](int e, float v) {
                if (r == 0) sRed[e] = v;
                else if (r < MW - 1) sRed[e] += v;
                else out[e] = sRed[e] + v;
            };
            for (int k = 0; k < NF; ++k) put(l * NF + k, g1[k]);
            put(o1 + l, gb1);
            for (int j = 0; j < NH; ++j) put(o2 + j * NH + l, g2[j]);
            put(o3 + l, gb2);
            for (int j = 0; j < KMAX; ++j)
                if (j < K) put(o4 + j * NH + l, g3[j]);
            if (l < K) put(o5 + l, gb3);
            if (l == 0) sLoss[r] = wl;
        }
        __syncthreads();
    }
    if (tid == 0) {
        double s = sLoss[0];
        for (int r = 1; r < MW; ++r) s += sLoss[r];
        lpart[blockIdx.x] = s;
    }
}

// Sum of the G partial gradients per parameter, in workgroup order, and the
// loss sum.  ADAM: the Adam update of the trainable parameters; otherwise the
// gradient is written out (zero on the standardisation block).
template <bool ADAM>
__global__ __launch_bounds__(256) void k_mlp_reduce(const float* __restrict__ part, int G, int ntr, int np,
                                                    const double* __restrict__ lpart, double* __restrict__ loss_sum,
                                                    float* __restrict__ grad, float* __restrict__ P,
                                                    float* __restrict__ M, float* __restrict__ V, float lr, float b1,
                                                    float b2, float eps, float c1, float c2) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t == 0 && loss_sum) {
        double s = 0.0;
        for (int g = 0; g < G; ++g) s += lpart[g];
        *loss_sum = s;
    }
    if (t >= np) return;
    if (t >= ntr) {
        if (!ADAM) grad[t] = 0.f;
        return;
    }
    float s = 0.f;
    int g = 0;
    for (; g + 8 <= G; g += 8) {
        float v[8];
        for (int u = 0; u < 8; ++u) v[u] = part[(size_t)(g + u) * ntr + t];
        for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; g < G; ++g) s += part[(size_t)g * ntr + t];
    if (!ADAM) {
        grad[t] = s;
        return;
    }
    const float m = b1 * M[t] + (1.f - b1) * s;
    const float v = b2 * V[t] + (1.f - b2) * s * s;
    M[t] = m;
    V[t] = v;
    P[t] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
}

// ---------------------------------------------------------------------------
// BF16 inference on the matrix cores.  Weights and activations are rounded to
// bfloat16 (nearest even), products accumulate in FP32
// (v_mfma_f32_16x16x16_bf16).  A wave takes 16 samples; each layer is computed
// transposed, units x samples = W (units x inputs) . A^T (inputs x samples),
// so a layer's accumulator registers (lane: sample l % 16, units 4 (l / 16)
// + i of a 16-unit block) are exactly the next layer's B operand.  The
// weights stay in registers as A operands for the whole launch.
// ---------------------------------------------------------------------------
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short bf16_bits(float x) {
    unsigned int u = __float_as_uint(x);
    if ((u & 0x7f800000u) != 0x7f800000u) u += 0x7fffu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

__global__ __launch_bounds__(256) void k_mlp_predict_bf16(const float* __restrict__ P, int K,
                                                          const float* __restrict__ X, int B, int* __restrict__ cls,
                                                          float* __restrict__ prob) {
    const int l = threadIdx.x & 63, c = l & 15, g = l >> 4;
    const float* W1 = P;
    const float* b1 = P + mlp_offsets(K, 1);
    const float* W2 = P + mlp_offsets(K, 2);
    const float* b2 = P + mlp_offsets(K, 3);
    const float* W3 = P + mlp_offsets(K, 4);
    const float* b3 = P + mlp_offsets(K, 5);
    const float* mu = P + mlp_offsets(K, 6);
    const float* sd = P + mlp_offsets(K, 7);
    // A operands: row (output unit) 16 mb + c, inputs 16 kb + 4 g + i
    bf16x4 w1a[4], w2a[4][4], w3a[4];
    f32x4 c1[4], c2[4], c3;
    for (int mb = 0; mb < 4; ++mb) {
        for (int i = 0; i < 4; ++i) {
            const int k = 4 * g + i;
            w1a[mb][i] = k < NF ? bf16_bits(W1[(mb * 16 + c) * NF + k]) : (short)0;
            c1[mb][i] = b1[mb * 16 + k];
            c2[mb][i] = b2[mb * 16 + k];
        }
        for (int kb = 0; kb < 4; ++kb)
            for (int i = 0; i < 4; ++i) w2a[mb][kb][i] = bf16_bits(W2[(mb * 16 + c) * NH + kb * 16 + 4 * g + i]);
    }
    for (int kb = 0; kb < 4; ++kb)
        for (int i = 0; i < 4; ++i) w3a[kb][i] = c < K ? bf16_bits(W3[c * NH + kb * 16 + 4 * g + i]) : (short)0;
    for (int i = 0; i < 4; ++i) c3[i] = 4 * g + i < K ? b3[4 * g + i] : 0.f;

    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6, nw = (gridDim.x * blockDim.x) >> 6;
    const int ntile = (B + 15) / 16;
    for (int t = wave; t < ntile; t += nw) {
        const int b = t * 16 + c;
        const bool ok = b < B;
        bf16x4 xb;
        for (int i = 0; i < 4; ++i) {
            const int k = 4 * g + i;
            xb[i] = (ok && k < NF) ? bf16_bits((X[(size_t)b * NF + k] - mu[k]) / sd[k]) : (short)0;
        }
        bf16x4 a1[4], a2[4];
        for (int mb = 0; mb < 4; ++mb) {
            const f32x4 h = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w1a[mb], xb, c1[mb], 0, 0, 0);
            for (int i = 0; i < 4; ++i) a1[mb][i] = bf16_bits(fmaxf(h[i], 0.f));
        }
        for (int mb = 0; mb < 4; ++mb) {
            f32x4 h = c2[mb];
            for (int kb = 0; kb < 4; ++kb) h = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w2a[mb][kb], a1[kb], h, 0, 0, 0);
            for (int i = 0; i < 4; ++i) a2[mb][i] = bf16_bits(fmaxf(h[i], 0.f));
        }
        f32x4 z = c3;
        for (int kb = 0; kb < 4; ++kb) z = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w3a[kb], a2[kb], z, 0, 0, 0);
        // lane (c, g) holds classes 4 g .. 4 g + 3 of sample c: the first
        // maximum over the four lanes of the sample
        float bv = -INFINITY;
        int bj = 0x7fffffff;
        for (int i = 0; i < 4; ++i)
            if (4 * g + i < K && z[i] > bv) {
                bv = z[i];
                bj = 4 * g + i;
            }
        for (int off = 16; off < 64; off <<= 1) {
            const float ov = __shfl_xor(bv, off, 64);
            const int oj = __shfl_xor(bj, off, 64);
            if (ov > bv || (ov == bv && oj < bj)) {
                bv = ov;
                bj = oj;
            }
        }
        if (ok && g == 0) cls[b] = bj;
        if (prob) {
            float e[4], s = 0.f;
            for (int i = 0; i < 4; ++i) {
                e[i] = 4 * g + i < K ? expf(z[i] - bv) : 0.f;
                s += e[i];
            }
            s += __shfl_xor(s, 16, 64);
            s += __shfl_xor(s, 32, 64);
            for (int i = 0; i < 4; ++i)
                if (ok && 4 * g + i < K) prob[(size_t)b * K + 4 * g + i] = e[i] / s;
        }
    }
}

// ---------------------------------------------------------------------------
// tail-mass check: reject a proposed level if any block its mask merges
// carries an indicator I_B = max(sum M1, sum M2) above C_split on the cell's
// distribution refined to V_base.  A wave takes up to TAIL_GROUP cells of one
// level, so the level's tables (the point holding each base point, the base
// weights, the point velocities) are read once for all of them.  The lanes
// walk V_base in 16 x 16-point tiles, one 2 x 2 block per lane in Morton
// order: the 4 x 4 and 8 x 8 blocks are runs of 4 and 16 lanes, summed by
// butterflies.  The totals are constants of the cell and a correctly rounded
// division is monotone, so max_B (m_B / T) = (max_B m_B) / T: one pass keeps
// the totals and the largest and smallest merged-block sums, and the decision
// is taken at the end.
// ---------------------------------------------------------------------------
template <typename S>
__global__ __launch_bounds__(256) void k_tail_check(const LevelDesc* __restrict__ lvs,
                                                    const int* __restrict__ cell_lev,
                                                    const int* __restrict__ cell_slot,
                                                    const int* __restrict__ groups, int n_groups,
                                                    const int* __restrict__ ptb_all, const int* __restrict__ ptb_off,
                                                    const uint8_t* __restrict__ kappa_all,
                                                    const int* __restrict__ pred, const double* __restrict__ bw,
                                                    int nx, int ny, double C_split, int* __restrict__ accept) {
    constexpr int G = TAIL_GROUP;
    const int lane = threadIdx.x & 63;
    const int gi = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + (threadIdx.x >> 6)));
    if (gi >= n_groups) return;
    const int nbx = nx / 2, nby = ny / 2, Nb = nbx * nby;
    int cell[G];
    for (int k = 0; k < G; ++k) cell[k] = groups[gi * G + k];     // -1: no cell
    const int lev = cell_lev[cell[0]];
    const LevelDesc& L = lvs[lev];
    const S* g[G];
    const S* h[G];
    const uint8_t* kp[G];
    for (int k = 0; k < G; ++k) {
        const int ck = cell[k] >= 0 ? cell[k] : cell[0];
        const size_t row = (size_t)cell_slot[ck] * L.stride;
        g[k] = reinterpret_cast<const S*>(L.g) + row;
        h[k] = reinterpret_cast<const S*>(L.h) + row;
        kp[k] = kappa_all + (size_t)pred[ck] * Nb;
    }
    const int* ptb = ptb_all + ptb_off[lev];
    const int mx = (lane & 1) | ((lane >> 1) & 2) | ((lane >> 2) & 4);
    const int my = ((lane >> 1) & 1) | ((lane >> 2) & 2) | ((lane >> 3) & 4);
    double T1[G], T2[G], hi1[G], lo1[G], hi2[G], lo2[G];
    for (int k = 0; k < G; ++k) {
        T1[k] = T2[k] = 0.0;
        hi1[k] = hi2[k] = -INFINITY;
        lo1[k] = lo2[k] = INFINITY;
    }
    const int ntx = (nx + 15) >> 4, nty = (ny + 15) >> 4;
    for (int t = 0; t < ntx * nty; ++t) {
        const int bx = (t % ntx) * 8 + mx, by = (t / ntx) * 8 + my;
        double a1[G], a2[G];
        for (int k = 0; k < G; ++k) a1[k] = a2[k] = 0.0;
        for (int d = 0; d < 4; ++d) {
            const int px = 2 * bx + (d & 1), py = 2 * by + (d >> 1);
            if (px < nx && py < ny) {
                const int b = px + nx * py;
                const int p = ptb[b];
                const double wb = bw[b], xp = L.xi_x[p], yp = L.xi_y[p];
                const double x2 = xp * xp + yp * yp;
                for (int k = 0; k < G; ++k) {
                    const double gp = (double)g[k][p];
                    a1[k] += wb * gp;
                    a2[k] += 0.5 * wb * ((double)h[k][p] + x2 * gp);
                }
            }
        }
        const bool blk = bx < nbx && by < nby;
        for (int k = 0; k < G; ++k) {
            T1[k] += a1[k];
            T2[k] += a2[k];
            const int s = blk ? kp[k][bx + nbx * by] : 0;
            const double m1 = blk ? a1[k] : 0.0, m2 = blk ? a2[k] : 0.0;
            double q1 = m1 + __shfl_xor(m1, 1, 64), q2 = m2 + __shfl_xor(m2, 1, 64);
            q1 += __shfl_xor(q1, 2, 64);
            q2 += __shfl_xor(q2, 2, 64);
            double r1 = q1 + __shfl_xor(q1, 4, 64), r2 = q2 + __shfl_xor(q2, 4, 64);
            r1 += __shfl_xor(r1, 8, 64);
            r2 += __shfl_xor(r2, 8, 64);
            if (s > 0) {
                const double v1 = s == 1 ? m1 : (s == 2 ? q1 : r1);
                const double v2 = s == 1 ? m2 : (s == 2 ? q2 : r2);
                hi1[k] = fmax(hi1[k], v1);
                lo1[k] = fmin(lo1[k], v1);
                hi2[k] = fmax(hi2[k], v2);
                lo2[k] = fmin(lo2[k], v2);
            }
        }
    }
    for (int k = 0; k < G; ++k)
        for (int off = 32; off > 0; off >>= 1) {
            T1[k] += __shfl_xor(T1[k], off, 64);
            T2[k] += __shfl_xor(T2[k], off, 64);
            hi1[k] = fmax(hi1[k], __shfl_xor(hi1[k], off, 64));
            lo1[k] = fmin(lo1[k], __shfl_xor(lo1[k], off, 64));
            hi2[k] = fmax(hi2[k], __shfl_xor(hi2[k], off, 64));
            lo2[k] = fmin(lo2[k], __shfl_xor(lo2[k], off, 64));
        }
    if (lane == 0)
        for (int k = 0; k < G; ++k) {
            if (cell[k] < 0) continue;
            const double A1 = (T1[k] >= 0.0 ? hi1[k] : lo1[k]) / T1[k];
            const double A2 = (T2[k] >= 0.0 ? hi2[k] : lo2[k]) / T2[k];
            accept[cell[k]] = (A1 > C_split || A2 > C_split) ? 0 : 1;
        }
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

size_t mlp_part_bytes(int B, int K) {
    return sizeof(float) * (size_t)mlp_groups(B) * (size_t)mlp_offsets(K, 6) + sizeof(double) * MAX_PART;
}

// part: mlp_part_bytes(B, K) bytes of device memory (partial gradients, then
// the per-workgroup loss sums)
static void split_part(void* part, int B, int K, float** pg, double** pl) {
    *pg = static_cast<float*>(part);
    *pl = reinterpret_cast<double*>(static_cast<char*>(part) + sizeof(float) * (size_t)mlp_groups(B) *
                                                                   (size_t)mlp_offsets(K, 6));
}

hipError_t launch_mlp_eval(hipStream_t st, const float* P, int K, const float* X, const int* y, int B, float* prob,
                           void* part, float* grad, double* loss_sum) {
    if (B < 1) return hipErrorInvalidValue;
    float* pg;
    double* pl;
    split_part(part, B, K, &pg, &pl);
    const int G = mlp_groups(B), ntr = mlp_offsets(K, 6), np = mlp_nparams(K);
    hipLaunchKernelGGL(k_mlp_batch<true>, dim3(G), dim3(256), 0, st, P, K, X, y, nullptr, B, prob, nullptr, pg, pl);
    hipLaunchKernelGGL(k_mlp_reduce<false>, dim3((np + 255) / 256), dim3(256), 0, st, pg, G, ntr, np, pl, loss_sum,
                       grad, nullptr, nullptr, nullptr, 0.f, 0.f, 0.f, 0.f, 1.f, 1.f);
    return hipGetLastError();
}

hipError_t launch_mlp_train_step(hipStream_t st, float* P, int K, const float* X, const int* y, const int* idx, int B,
                                 void* part, double* loss_sum, float* M, float* V, float lr, float b1, float b2,
                                 float eps, int t) {
    float* pg;
    double* pl;
    split_part(part, B, K, &pg, &pl);
    const int G = mlp_groups(B), ntr = mlp_offsets(K, 6);
    const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    hipLaunchKernelGGL(k_mlp_batch<true>, dim3(G), dim3(256), 0, st, P, K, X, y, idx, B, nullptr, nullptr, pg, pl);
    hipLaunchKernelGGL(k_mlp_reduce<true>, dim3((ntr + 255) / 256), dim3(256), 0, st, pg, G, ntr, ntr, pl, loss_sum,
                       nullptr, P, M, V, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// forward/backward without device allocation: the partial gradients live in a
// fixed device array of the library
// ---------------------------------------------------------------------------
// Layout (bytes): [0, 256) the loss sum when the caller wants none; then the
// partial gradients and loss sums of at most MAX_PART workgroups (a batch of
// at most NOALLOC_MAX_BATCH samples needs no more).  Each GPU holds its own
// copy until the process ends; calls on one GPU share it.
static_assert((NOALLOC_MAX_BATCH + CHUNK - 1) / CHUNK <= MAX_PART, "no-allocation batch limit");
constexpr size_t NOALLOC_BYTES = 256 + sizeof(float) * (size_t)MAX_PART * NTR_MAX + sizeof(double) * MAX_PART;
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

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
    if (mlp_part_bytes(B, K) > NOALLOC_BYTES - 256) return hipErrorInvalidValue;
    if (grad) return launch_mlp_eval(st, P, K, X, y, B, prob, base + 256, grad, ls);
    // no gradient wanted: the partials are formed and left in the array
    float* pg;
    double* pl;
    split_part(base + 256, B, K, &pg, &pl);
    const int G = mlp_groups(B), ntr = mlp_offsets(K, 6);
    hipLaunchKernelGGL(k_mlp_batch<true>, dim3(G), dim3(256), 0, st, P, K, X, y, nullptr, B, prob, nullptr, pg, pl);
    hipLaunchKernelGGL(k_mlp_reduce<false>, dim3(1), dim3(64), 0, st, pg, G, ntr, 0, pl, ls, nullptr, nullptr,
                       nullptr, nullptr, 0.f, 0.f, 0.f, 0.f, 1.f, 1.f);
    return hipGetLastError();
}

hipError_t launch_mlp_predict(hipStream_t st, const float* P, int K, const float* X, int B, int bf16, int* cls,
                              float* prob) {
    if (B <= 0) return hipSuccess;
    if (bf16) {
        const int waves = (B + 15) / 16;
        const int wg = std::min((waves + 3) / 4, 2048);
        hipLaunchKernelGGL(k_mlp_predict_bf16, dim3(wg), dim3(256), 0, st, P, K, X, B, cls, prob);
    } else {
        const int wg = std::min((B + CHUNK - 1) / CHUNK, 4096);
        hipLaunchKernelGGL(k_mlp_batch<false>, dim3(wg), dim3(256), 0, st, P, K, X, nullptr, nullptr, B, prob, cls,
                           nullptr, nullptr);
    }
    return hipGetLastError();
}

hipError_t launch_tail_check(int prec, hipStream_t st, const LevelDesc* lv, const int* cell_lev, const int* cell_slot,
                             const int* groups, int n_groups, const int* ptb_all, const int* ptb_off,
                             const uint8_t* kappa_all, const int* pred, const double* bw, int nx, int ny,
                             double C_split, int* accept) {
    if (n_groups <= 0) return hipSuccess;
    const dim3 grid((n_groups + 3) / 4);
    if (prec == 32)
        hipLaunchKernelGGL(k_tail_check<float>, grid, dim3(256), 0, st, lv, cell_lev, cell_slot, groups, n_groups,
                           ptb_all, ptb_off, kappa_all, pred, bw, nx, ny, C_split, accept);
    else
        hipLaunchKernelGGL(k_tail_check<double>, grid, dim3(256), 0, st, lv, cell_lev, cell_slot, groups, n_groups,
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
