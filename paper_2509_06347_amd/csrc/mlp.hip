/*
 * Warm-start surrogate: a 5 -> 256 -> 256 -> 256 -> 4 MLP with SiLU, trained
 * and evaluated with BF16 matrix-core (MFMA) GEMMs and FP32 accumulation.
 *
 * Master weights, biases and Adam moments are FP32; every GEMM reads BF16
 * copies of weights and activations.  Weights follow y = x W^T + b with W
 * stored [out][in] (in padded to a multiple of 32).  The inputs are the
 * standardised features (Mach, log10 Re, x, y, wall distance); the outputs the
 * standardised targets (log rho, u/U_inf, v/U_inf, log p).
 *
 * GEMM: C[M x N] = A[M x K] B[K x N] with arbitrary strides, one 64 x 64 block
 * tile per 256-thread block (four wave64s, each 32 x 32 = 2 x 2 MFMA tiles of
 * v_mfma_f32_16x16x32_bf16), K staged through LDS in steps of 32; operands
 * with a unit stride along k or along their rows are loaded 16 bytes per
 * thread (the training step's GEMMs all are).
 * Fragment layout of the 16x16x32 BF16 MFMA: lane l holds A row (l % 16) and
 * B column (l % 16), each with the 8 consecutive K values 8 * (l / 16) ..;
 * the accumulator holds column (l % 16), rows 4 * (l / 16) .. + 3.
 */
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <random>
#include <vector>

#include "cgks_internal.h"

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int NL = 4;                                  /* layers */
constexpr int DIN[NL] = {5, 256, 256, 256};
constexpr int DOUT[NL] = {256, 256, 256, 4};
constexpr int KPAD[NL] = {32, 256, 256, 256};          /* padded input width */
constexpr int NPAD[NL] = {256, 256, 256, 16};          /* padded output width */

enum { EPI_STORE = 0, EPI_BIAS_SILU = 1, EPI_BIAS = 2, EPI_DSILU = 3, EPI_BIAS_SILU_NOZ = 4 };

__device__ __forceinline__ float silu_f(float z) { return z / (1.0f + __expf(-z)); }
__device__ __forceinline__ float dsilu_f(float z) {
    const float s = 1.0f / (1.0f + __expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

/*
 * C = A B (+ epilogue).  A(m,k) = A[m*sam + k*sak], B(k,n) = B[k*sbk + n*sbn].
 * EPI_BIAS_SILU: Z = C + bias[n] -> Cz (fp32) and Cb = bf16(silu(Z)).
 * EPI_BIAS_SILU_NOZ: Cb = bf16(silu(C + bias[n])) only (inference).
 * EPI_BIAS:      C + bias[n] -> C (fp32).
 * EPI_DSILU:     Cb = bf16(C * silu'(Zin[m, n]))  (backward through SiLU).
 * EPI_STORE:     C -> C (fp32).
 * Block z of the grid's third dimension sums k in [z kc, min(K, (z + 1) kc))
 * and, for EPI_STORE, writes to Cz + z zstride (split-K partials).
 * Out-of-range A/B elements read as zero; only in-range C elements are stored.
 */
/* Operand layouts for the tile loader: X(r, k) = X[r * srow + k * sk]. */
enum { LAY_ANY = 0, LAY_K = 1, LAY_R = 2 };   /* any strides; k contiguous; r contiguous */

/* Stage a 64 x 32 (rows x k) tile of X into Xs[r][k] (zeros outside [0, R) x
 * [k0, ke)).  LAY_K: each thread loads 8 consecutive k of one row (16 bytes);
 * LAY_R: 8 consecutive rows of one k (16 bytes), transposed into LDS; both
 * need 16-byte aligned rows / columns, which the host checks.  LAY_ANY: one
 * element at a time. */
template <int LAY>
__device__ __forceinline__ void load_tile(__bf16 (*Xs)[40], const __bf16* __restrict__ X, long srow, long sk, int r0,
                                          int R, int k0, int ke, int t) {
    if constexpr (LAY == LAY_K) {
        const int r = t >> 2, kc = (t & 3) * 8, gr = r0 + r, gk = k0 + kc;
        if (gr < R && gk + 8 <= ke) {
            *reinterpret_cast<uint4*>(&Xs[r][kc]) = *reinterpret_cast<const uint4*>(X + (long)gr * srow + gk);
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e)
                Xs[r][kc + e] = (gr < R && gk + e < ke) ? X[(long)gr * srow + gk + e] : (__bf16)0.0f;
        }
    } else if constexpr (LAY == LAY_R) {
        const int kk = t >> 3, rc = (t & 7) * 8, gr = r0 + rc, gk = k0 + kk;
        bf16x8 v;
        if (gk < ke && gr + 8 <= R) {
            v = *reinterpret_cast<const bf16x8*>(X + gr + (long)gk * sk);
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = (gk < ke && gr + e < R) ? X[gr + e + (long)gk * sk] : (__bf16)0.0f;
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) Xs[rc + e][kk] = v[e];
    } else {
        const int r = t >> 2, kc = (t & 3) * 8, gr = r0 + r;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = k0 + kc + e;
            Xs[r][kc + e] = (gr < R && k < ke) ? X[(long)gr * srow + (long)k * sk] : (__bf16)0.0f;
        }
    }
}

template <int EPI, int LA, int LB>
__global__ void __launch_bounds__(256) k_gemm(int M, int N, int K, const __bf16* __restrict__ A, long sam, long sak,
                                              const __bf16* __restrict__ B, long sbk, long sbn, float* Cz, long ldc,
                                              __bf16* Cb, long ldb, const float* bias, const float* Zin, long ldz,
                                              int kc, long zstride) {
    __shared__ __attribute__((aligned(16))) __bf16 As[64][40];   /* [m][k], padded rows (80 bytes) */
    __shared__ __attribute__((aligned(16))) __bf16 Bs[64][40];   /* [n][k] */
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
    const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int kb = blockIdx.z * kc, ke = min(K, kb + kc);
    if (EPI == EPI_STORE) Cz += blockIdx.z * zstride;
    for (int k0 = kb; k0 < ke; k0 += 32) {
        load_tile<LA>(As, A, sam, sak, m0, M, k0, ke, t);
        load_tile<LB>(Bs, B, sbn, sbk, n0, N, k0, ke, t);
        __syncthreads();
        const int fr = lane & 15, fk = (lane >> 4) * 8;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            bf16x8 a;
#pragma unroll
            for (int e = 0; e < 8; ++e) a[e] = As[wm + 16 * i + fr][fk + e];
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                bf16x8 b;
#pragma unroll
                for (int e = 0; e < 8; ++e) b[e] = Bs[wn + 16 * j + fr][fk + e];
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[i][j], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    const int cc = lane & 15, cr = (lane >> 4) * 4;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm + 16 * i + cr + r, n = n0 + wn + 16 * j + cc;
                if (m >= M || n >= N) continue;
                float v = acc[i][j][r];
                if (EPI == EPI_BIAS_SILU) {
                    v += bias[n];
                    Cz[(long)m * ldc + n] = v;
                    Cb[(long)m * ldb + n] = (__bf16)silu_f(v);
                } else if (EPI == EPI_BIAS_SILU_NOZ) {
                    Cb[(long)m * ldb + n] = (__bf16)silu_f(v + bias[n]);
                } else if (EPI == EPI_BIAS) {
                    Cz[(long)m * ldc + n] = v + bias[n];
                } else if (EPI == EPI_DSILU) {
                    Cb[(long)m * ldb + n] = (__bf16)(v * dsilu_f(Zin[(long)m * ldz + n]));
                } else {
                    Cz[(long)m * ldc + n] = v;
                }
            }
}

/* C[i] = sum_z P[z][i] in increasing z (fixed order). */
__global__ void k_splitk_reduce(const float* P, int nz, long cnt, float* C) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cnt) return;
    float v = 0.0f;
    for (int z = 0; z < nz; ++z) v += P[z * cnt + i];
    C[i] = v;
}

/* Features [n][5] (fp32) -> bf16 [n][32] zero-padded. */
__global__ void k_pack_input(const float* X, __bf16* H, int n) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * 32) return;
    const int i = t >> 5, k = t & 31;
    H[t] = (k < 5) ? (__bf16)X[i * 5 + k] : (__bf16)0.0f;
}

/* Output gradient 2 (out - Y) / n as bf16 [n][16] zero-padded, and per-sample squared error. */
__global__ void k_out_grad(const float* out, const float* Y, __bf16* G, float* se, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float s = 0.0f;
    for (int k = 0; k < 16; ++k) {
        float g = 0.0f;
        if (k < 4) {
            const float d = out[i * 16 + k] - Y[i * 4 + k];
            s += d * d;
            g = 2.0f * d / (float)n;
        }
        G[i * 16 + k] = (__bf16)g;
    }
    se[i] = s;
}

/* Column sums of a [n][ncol] bf16 matrix in a fixed order (bias gradients). */
/* Column sums of G [n][ld] (bf16), columns 0..ncol-1, in two fixed-order
 * passes: block b sums rows [b R, (b + 1) R) of every column (consecutive
 * threads read consecutive columns of a row; the row loads are unrolled so
 * they are in flight together), then one block per column reduces the block
 * partials in a fixed tree. */
constexpr int CS_ROWS = 64;
__global__ void k_colsum_part(const __bf16* G, int n, int ld, int ncol, float* part) {
    const int c = threadIdx.x, b = blockIdx.x;
    if (c >= ncol) return;
    const int i0 = b * CS_ROWS;
    float v = 0.0f;
#pragma unroll 16
    for (int r = 0; r < CS_ROWS; ++r) {
        const int i = i0 + r;
        v += i < n ? (float)G[(long)i * ld + c] : 0.0f;
    }
    part[(long)b * ncol + c] = v;
}

__global__ void k_colsum_final(const float* part, int nb, int ncol, float* out) {
    const int c = blockIdx.x;
    __shared__ float sh[256];
    float v = 0.0f;
    for (int b = threadIdx.x; b < nb; b += 256) v += part[(long)b * ncol + c];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = sh[0];
}

/* Mean of a[0..n): 256-element blocks reduced in a fixed tree order, then the
 * block sums added in block order by one block. */
__global__ void k_sum_part(const float* a, int n, float* part) {
    __shared__ float sh[256];
    const int i = blockIdx.x * 256 + threadIdx.x;
    sh[threadIdx.x] = i < n ? a[i] : 0.0f;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void k_sum(const float* a, int n, float* out, int count) {
    __shared__ float sh[256];
    float v = 0.0f;
    for (int i = threadIdx.x; i < n; i += 256) v += a[i];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0] / (float)count;
}

/* Adam on fp32 master parameters; refreshes the bf16 weight copy (bias: wb null). */
__global__ void k_adam(float* p, const float* g, float* m, float* v, __bf16* wb, int cnt, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= cnt) return;
    const float gi = g[t];
    const float mi = b1 * m[t] + (1.0f - b1) * gi;
    const float vi = b2 * v[t] + (1.0f - b2) * gi * gi;
    m[t] = mi;
    v[t] = vi;
    const float pn = p[t] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    p[t] = pn;
    if (wb) wb[t] = (__bf16)pn;
}

__global__ void k_to_bf16(const float* a, __bf16* b, int cnt) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < cnt) b[t] = (__bf16)a[t];
}

/* Raw features of every fine cell [n][5]: Mach, log10 Re, centroid x and y
 * (SoA centroids C [2][n]) and the distance to the nearest wall-face centre
 * (wc [nw][2]; 0 without walls).  The one definition used both to build
 * training data and to evaluate the network for a warm start. */
__global__ void k_features(const double* C, int n, const double* wc, int nw, double mach, double lre, float* X) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double x = C[i], y = C[n + i];
    double d2 = nw > 0 ? 1e300 : 0.0;
    for (int k = 0; k < nw; ++k) {
        const double dx = x - wc[2 * k], dy = y - wc[2 * k + 1];
        d2 = fmin(d2, dx * dx + dy * dy);
    }
    float* o = X + (size_t)i * 5;
    o[0] = (float)mach;
    o[1] = (float)lre;
    o[2] = (float)x;
    o[3] = (float)y;
    o[4] = (float)sqrt(d2);
}

/* Standardised features (X - mean) / std in place; a cell whose features lie
 * outside the training range [lo, hi] (when a range is set) is marked for the
 * free-stream fallback. */
__global__ void k_standardise(float* X, int n, const float* mean_std, const float* range, int* out_of_range) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    bool out = false;
    for (int k = 0; k < 5; ++k) {
        const float v = X[(size_t)i * 5 + k];
        if (range && (v < range[k] || v > range[5 + k])) out = true;
        X[(size_t)i * 5 + k] = (v - mean_std[k]) / mean_std[5 + k];
    }
    out_of_range[i] = out ? 1 : 0;
}

/* Network output -> conservative state [n][D+2] (AoS), with a free-stream fallback per cell. */
template <int D>
__global__ void k_mlp_state(const float* out, const float* tt, double mach, double gamma, const double* uinf, double* W,
                            int n, int* fallback, const int* out_of_range) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double y[4];
    for (int k = 0; k < 4; ++k) y[k] = (double)out[i * 16 + k] * (double)tt[4 + k] + (double)tt[k];
    const double rho = exp(y[0]), u = y[1] * mach, v = y[2] * mach, p = exp(y[3]) / gamma;
    const bool ok = !out_of_range[i] && isfinite(rho) && isfinite(u) && isfinite(v) && isfinite(p) && rho > 1e-6 &&
                    p > 1e-8 && rho < 1e4 && p < 1e6;
    double r = rho, U[3] = {u, v, 0.0}, pr = p;
    if (!ok) {
        atomicAdd(fallback, 1);
        r = 1.0;
        pr = 1.0 / gamma;
        for (int d = 0; d < 3; ++d) U[d] = uinf[d];
    }
    double ke = 0.0;
    double* w = W + (long)i * (D + 2);
    w[0] = r;
    for (int d = 0; d < D; ++d) {
        w[1 + d] = r * U[d];
        ke += U[d] * U[d];
    }
    w[D + 1] = pr / (gamma - 1.0) + 0.5 * r * ke;
}

inline int nb(long m, int b) { return (int)((m + b - 1) / b); }

/* Fixed workspace of cgks_mlp_forward_noalloc: for CGKS_MLP_NOALLOC_MAX_ROWS
 * rows, the packed input (32 bf16 per row) then two ping-pong hidden layers
 * (256 bf16 per row each); 17.8 MB per device, held until the process ends. */
constexpr size_t NOALLOC_H0 = 0;
constexpr size_t NOALLOC_HA = (size_t)CGKS_MLP_NOALLOC_MAX_ROWS * 32;
constexpr size_t NOALLOC_HB = NOALLOC_HA + (size_t)CGKS_MLP_NOALLOC_MAX_ROWS * 256;
constexpr size_t NOALLOC_ELEMS = NOALLOC_HB + (size_t)CGKS_MLP_NOALLOC_MAX_ROWS * 256;

}  // namespace

static __device__ __align__(256) __bf16 scratch[NOALLOC_ELEMS];

namespace {

/* Device address of `scratch` on the current device.  In host code the
 * array's name is only a host-side stand-in, so kernels are given this
 * address, looked up once per device. */
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
__bf16* g_scratch_ptr[MAX_DEVICES] = {};

int scratch_address(__bf16** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return CGKS_EDEVICE;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return CGKS_EDEVICE;
        g_scratch_ptr[dev] = (__bf16*)p;
    }
    *out = g_scratch_ptr[dev];
    return CGKS_OK;
}

}  // namespace

struct cgks_mlp {
    float* P[NL][2];            /* master W [NPAD?] -> stored [DOUT][KPAD], bias [DOUT] */
    float *Mo[NL][2], *Vo[NL][2], *Gr[NL][2];
    __bf16* Wb[NL];             /* bf16 copy of W, [DOUT][KPAD] */
    int t = 0;
    int cap = 0;                /* samples the workspace holds */
    size_t part_cnt = 0;        /* floats in part */
    __bf16* H[NL];              /* layer inputs (bf16), [cap][KPAD] */
    float* Z[NL];               /* pre-activations (fp32), [cap][NPAD] */
    float* out;                 /* [cap][16] */
    __bf16* G[NL + 1];          /* gradients w.r.t. layer outputs, bf16 */
    float* se;                  /* per-sample squared error */
    float* dloss;
    float* part;                /* split-K partials (SPLITK * 256 * 256) and bias-gradient block sums */
    hipStream_t stream = nullptr;
    std::vector<void*> allocs;
    std::string err;
    bool have_range = false;
    float range[10];            /* training range of the raw features: lo [5], hi [5] */
};

namespace {

template <class T>
hipError_t mal(cgks_mlp* m, T** p, size_t cnt) {
    hipError_t e = hipMalloc((void**)p, (cnt ? cnt : 1) * sizeof(T));
    if (e == hipSuccess) m->allocs.push_back((void*)*p);
    return e;
}

size_t wcount(int l) { return (size_t)DOUT[l] * KPAD[l]; }

int ensure_ws(cgks_mlp* m, int n) {
    if (n <= m->cap) return CGKS_OK;
    int cap = std::max(n, 2 * m->cap);
    bool ok = true;
    for (int l = 0; l < NL; ++l) {
        ok &= mal(m, &m->H[l], (size_t)cap * KPAD[l]) == hipSuccess;
        ok &= mal(m, &m->Z[l], (size_t)cap * NPAD[l]) == hipSuccess;
    }
    ok &= mal(m, &m->out, (size_t)cap * 16) == hipSuccess;
    for (int l = 0; l <= NL; ++l) ok &= mal(m, &m->G[l], (size_t)cap * (l < NL ? KPAD[l] : 16)) == hipSuccess;
    ok &= mal(m, &m->se, (size_t)cap) == hipSuccess;
    /* the partial buffer also holds the bias-gradient block sums, n / 64 x 256 */
    const size_t need = ((size_t)cap / CS_ROWS + 1) * 256;
    if (ok && need > m->part_cnt) {
        ok &= mal(m, &m->part, need) == hipSuccess;
        if (ok) m->part_cnt = need;
    }
    if (!ok) return CGKS_EDEVICE;
    m->cap = cap;
    return CGKS_OK;
}

/* Loader layout of an operand X(r, k) = X[r * srow + k * sk]: 16-byte vector
 * loads need a unit stride along k (or r) and 16-byte aligned rows (columns). */
int layout(const __bf16* X, long srow, long sk) {
    const bool al = reinterpret_cast<uintptr_t>(X) % 16 == 0;
    if (al && sk == 1 && srow % 8 == 0) return LAY_K;
    if (al && srow == 1 && sk % 8 == 0) return LAY_R;
    return LAY_ANY;
}

template <int EPI, int LA, int LB>
void launch_gemm(hipStream_t st, dim3 grid, int M, int N, int K, const __bf16* A, long sam, long sak, const __bf16* B,
                 long sbk, long sbn, float* Cz, long ldc, __bf16* Cb, long ldb, const float* bias, const float* Zin,
                 long ldz, int kc, long zs) {
    k_gemm<EPI, LA, LB><<<grid, 256, 0, st>>>(M, N, K, A, sam, sak, B, sbk, sbn, Cz, ldc, Cb, ldb, bias, Zin, ldz, kc,
                                              zs);
}

template <int EPI, int LA>
void dispatch_b(int lb, hipStream_t st, dim3 grid, int M, int N, int K, const __bf16* A, long sam, long sak,
                const __bf16* B, long sbk, long sbn, float* Cz, long ldc, __bf16* Cb, long ldb, const float* bias,
                const float* Zin, long ldz, int kc, long zs) {
    if (lb == LAY_K)
        launch_gemm<EPI, LA, LAY_K>(st, grid, M, N, K, A, sam, sak, B, sbk, sbn, Cz, ldc, Cb, ldb, bias, Zin, ldz, kc, zs);
    else if (lb == LAY_R)
        launch_gemm<EPI, LA, LAY_R>(st, grid, M, N, K, A, sam, sak, B, sbk, sbn, Cz, ldc, Cb, ldb, bias, Zin, ldz, kc, zs);
    else
        launch_gemm<EPI, LA, LAY_ANY>(st, grid, M, N, K, A, sam, sak, B, sbk, sbn, Cz, ldc, Cb, ldb, bias, Zin, ldz, kc,
                                      zs);
}

template <int EPI>
void gemm_any(hipStream_t st, dim3 grid, int M, int N, int K, const __bf16* A, long sam, long sak, const __bf16* B,
              long sbk, long sbn, float* Cz, long ldc, __bf16* Cb, long ldb, const float* bias, const float* Zin,
              long ldz, int kc, long zs) {
    const int la = layout(A, sam, sak), lb = layout(B, sbn, sbk);
    if (la == LAY_K)
        dispatch_b<EPI, LAY_K>(lb, st, grid, M, N, K, A, sam, sak, B, sbk, sbn, Cz, ldc, Cb, ldb, bias, Zin, ldz, kc, zs);
    else if (la == LAY_R)
        dispatch_b<EPI, LAY_R>(lb, st, grid, M, N, K, A, sam, sak, B, sbk, sbn, Cz, ldc, Cb, ldb, bias, Zin, ldz, kc, zs);
    else
        dispatch_b<EPI, LAY_ANY>(lb, st, grid, M, N, K, A, sam, sak, B, sbk, sbn, Cz, ldc, Cb, ldb, bias, Zin, ldz, kc,
                                 zs);
}

template <int EPI>
void gemm(hipStream_t st, int M, int N, int K, const __bf16* A, long sam, long sak, const __bf16* B, long sbk, long sbn,
          float* Cz, long ldc, __bf16* Cb, long ldb, const float* bias, const float* Zin, long ldz) {
    dim3 grid(nb(N, 64), nb(M, 64), 1);
    gemm_any<EPI>(st, grid, M, N, K, A, sam, sak, B, sbk, sbn, Cz, ldc, Cb, ldb, bias, Zin, ldz, K, 0);
}

/* C[M][N] (ldc == N) = A B with the K range split over up to SPLITK blocks;
 * the partials are summed in a fixed order, so the result is reproducible. */
constexpr int SPLITK = 64;
void gemm_splitk(cgks_mlp* m, int M, int N, int K, const __bf16* A, long sam, long sak, const __bf16* B, long sbk,
                 long sbn, float* C);

void gemm_splitk(cgks_mlp* m, int M, int N, int K, const __bf16* A, long sam, long sak, const __bf16* B, long sbk,
                 long sbn, float* C) {
    const int nz = std::max(1, std::min(SPLITK, K / 256));   /* >= 8 k-steps of 32 per block */
    const int kc = ((K + nz - 1) / nz + 31) / 32 * 32;
    const int z = (K + kc - 1) / kc;
    dim3 grid(nb(N, 64), nb(M, 64), z);
    const long cnt = (long)M * N;
    gemm_any<EPI_STORE>(m->stream, grid, M, N, K, A, sam, sak, B, sbk, sbn, m->part, N, nullptr, 0, nullptr, nullptr, 0,
                        kc, cnt);
    k_splitk_reduce<<<nb(cnt, 256), 256, 0, m->stream>>>(m->part, z, cnt, C);
}

/* forward of n samples (X device fp32 [n][5]) into m->out [n][16] */
void forward(cgks_mlp* m, const float* X, int n) {
    hipStream_t st = m->stream;
    k_pack_input<<<nb((long)n * 32, 256), 256, 0, st>>>(X, m->H[0], n);
    for (int l = 0; l < NL; ++l) {
        /* Z = H W^T + b : A = H [n][KPAD], B(k, o) = W[o][k] */
        if (l < NL - 1)
            gemm<EPI_BIAS_SILU>(st, n, DOUT[l], KPAD[l], m->H[l], KPAD[l], 1, m->Wb[l], 1, KPAD[l], m->Z[l], NPAD[l],
                                m->H[l + 1], KPAD[l + 1], m->P[l][1], nullptr, 0);
        else
            gemm<EPI_BIAS>(st, n, DOUT[l], KPAD[l], m->H[l], KPAD[l], 1, m->Wb[l], 1, KPAD[l], m->out, 16, nullptr, 0,
                           m->P[l][1], nullptr, 0);
    }
}

/* gradients of the mean squared error into m->Gr, loss into m->dloss */
void backward(cgks_mlp* m, const float* Y, int n) {
    hipStream_t st = m->stream;
    k_out_grad<<<nb(n, 256), 256, 0, st>>>(m->out, Y, m->G[NL], m->se, n);
    const int nbs = nb(n, 256);
    k_sum_part<<<nbs, 256, 0, st>>>(m->se, n, m->part);
    k_sum<<<1, 256, 0, st>>>(m->part, nbs, m->dloss, n);
    for (int l = NL - 1; l >= 0; --l) {
        const int ldg = (l == NL - 1) ? 16 : KPAD[l + 1];  /* row stride of the output gradient */
        /* dW[o][k] = sum_i G[i][o] H[i][k] : A(o, i) = G[i][o], B(i, k) = H[i][k] */
        gemm_splitk(m, DOUT[l], KPAD[l], n, m->G[l + 1], 1, ldg, m->H[l], KPAD[l], 1, m->Gr[l][0]);
        {
            /* bias gradient: column sums of the output gradient, through the
             * split-K partial buffer (free again once the reduce above ran;
             * n / 64 blocks x 256 columns fit it for every n the workspace
             * holds) */
            const int nch = nb(n, CS_ROWS);
            k_colsum_part<<<nch, 256, 0, st>>>(m->G[l + 1], n, ldg, DOUT[l], m->part);
            k_colsum_final<<<DOUT[l], 256, 0, st>>>(m->part, nch, DOUT[l], m->Gr[l][1]);
        }
        if (l > 0) {
            /* G_l[i][k] = (sum_o G[i][o] W[o][k]) * silu'(Z_{l-1}[i][k]) */
            gemm<EPI_DSILU>(st, n, DIN[l], DOUT[l], m->G[l + 1], ldg, 1, m->Wb[l], KPAD[l], 1, nullptr, 0, m->G[l],
                            KPAD[l], nullptr, m->Z[l - 1], NPAD[l - 1]);
        }
    }
}

}  // namespace

extern "C" {

int cgks_mlp_create(cgks_mlp** out, int seed) {
    if (!out) return CGKS_EINVAL;
    cgks_mlp* m = new cgks_mlp();
    std::mt19937_64 rng((uint64_t)seed);
    bool ok = mal(m, &m->dloss, 1) == hipSuccess && mal(m, &m->part, (size_t)SPLITK * 256 * 256) == hipSuccess;
    m->part_cnt = (size_t)SPLITK * 256 * 256;
    for (int l = 0; l < NL && ok; ++l) {
        const size_t nw = wcount(l), nbias = DOUT[l];
        std::vector<float> W(nw, 0.0f), b(nbias, 0.0f);
        const double bound = std::sqrt(6.0 / DIN[l]);
        std::uniform_real_distribution<double> U(-bound, bound);
        for (int o = 0; o < DOUT[l]; ++o)
            for (int k = 0; k < DIN[l]; ++k) W[(size_t)o * KPAD[l] + k] = (float)U(rng);
        for (int j = 0; j < 2 && ok; ++j) {
            const size_t cnt = j ? nbias : nw;
            ok &= mal(m, &m->P[l][j], cnt) == hipSuccess && mal(m, &m->Mo[l][j], cnt) == hipSuccess &&
                  mal(m, &m->Vo[l][j], cnt) == hipSuccess && mal(m, &m->Gr[l][j], cnt) == hipSuccess;
            if (!ok) break;
            ok &= hipMemcpy(m->P[l][j], j ? b.data() : W.data(), cnt * 4, hipMemcpyHostToDevice) == hipSuccess;
            ok &= hipMemset(m->Mo[l][j], 0, cnt * 4) == hipSuccess && hipMemset(m->Vo[l][j], 0, cnt * 4) == hipSuccess;
        }
        ok &= mal(m, &m->Wb[l], nw) == hipSuccess;
        if (ok) k_to_bf16<<<nb(nw, 256), 256>>>(m->P[l][0], m->Wb[l], (int)nw);
    }
    __bf16* ws = nullptr;
    if (!ok || hipDeviceSynchronize() != hipSuccess || scratch_address(&ws) != CGKS_OK) {
        cgks_mlp_destroy(m);
        return CGKS_EDEVICE;
    }
    *out = m;
    return CGKS_OK;
}

void cgks_mlp_destroy(cgks_mlp* m) {
    if (!m) return;
    (void)hipDeviceSynchronize();
    for (void* p : m->allocs) (void)hipFree(p);
    delete m;
}

int cgks_mlp_set_stream(cgks_mlp* m, void* stream) {
    if (!m) return CGKS_EINVAL;
    m->stream = (hipStream_t)stream;
    return CGKS_OK;
}

int cgks_mlp_num_params(void) {
    int s = 0;
    for (int l = 0; l < NL; ++l) s += DOUT[l] * DIN[l] + DOUT[l];
    return s;
}

/* Flat host layout: for each layer W [out][in] (unpadded) then b [out]. */
int cgks_mlp_get_weights(cgks_mlp* m, float* flat) {
    if (!m || !flat) return CGKS_EINVAL;
    size_t o = 0;
    for (int l = 0; l < NL; ++l) {
        std::vector<float> W(wcount(l));
        if (hipMemcpy(W.data(), m->P[l][0], W.size() * 4, hipMemcpyDeviceToHost) != hipSuccess) return CGKS_EDEVICE;
        for (int r = 0; r < DOUT[l]; ++r)
            for (int k = 0; k < DIN[l]; ++k) flat[o++] = W[(size_t)r * KPAD[l] + k];
        if (hipMemcpy(flat + o, m->P[l][1], DOUT[l] * 4, hipMemcpyDeviceToHost) != hipSuccess) return CGKS_EDEVICE;
        o += DOUT[l];
    }
    return CGKS_OK;
}

int cgks_mlp_set_weights(cgks_mlp* m, const float* flat) {
    if (!m || !flat) return CGKS_EINVAL;
    size_t o = 0;
    for (int l = 0; l < NL; ++l) {
        std::vector<float> W(wcount(l), 0.0f);
        for (int r = 0; r < DOUT[l]; ++r)
            for (int k = 0; k < DIN[l]; ++k) W[(size_t)r * KPAD[l] + k] = flat[o++];
        if (hipMemcpy(m->P[l][0], W.data(), W.size() * 4, hipMemcpyHostToDevice) != hipSuccess) return CGKS_EDEVICE;
        if (hipMemcpy(m->P[l][1], flat + o, DOUT[l] * 4, hipMemcpyHostToDevice) != hipSuccess) return CGKS_EDEVICE;
        o += DOUT[l];
        k_to_bf16<<<nb(wcount(l), 256), 256, 0, m->stream>>>(m->P[l][0], m->Wb[l], (int)wcount(l));
        (void)hipMemset(m->Mo[l][0], 0, wcount(l) * 4);
        (void)hipMemset(m->Vo[l][0], 0, wcount(l) * 4);
        (void)hipMemset(m->Mo[l][1], 0, DOUT[l] * 4);
        (void)hipMemset(m->Vo[l][1], 0, DOUT[l] * 4);
    }
    m->t = 0;
    return hipStreamSynchronize(m->stream) == hipSuccess ? CGKS_OK : CGKS_EDEVICE;
}

int cgks_mlp_forward(cgks_mlp* m, const float* X, float* Y, int n) {
    if (!m || n < 0) return CGKS_EINVAL;
    if (n == 0) return CGKS_OK;
    if (!X || !Y) return CGKS_EINVAL;
    int rc = ensure_ws(m, n);
    if (rc) return rc;
    forward(m, X, n);
    if (hipMemcpy2DAsync(Y, 4 * sizeof(float), m->out, 16 * sizeof(float), 4 * sizeof(float), n,
                         hipMemcpyDeviceToDevice, m->stream) != hipSuccess)
        return CGKS_EDEVICE;
    return hipStreamSynchronize(m->stream) == hipSuccess ? CGKS_OK : CGKS_EDEVICE;
}

int cgks_mlp_forward_noalloc(cgks_mlp* m, const float* X, float* Y, int n) {
    if (!m || n < 0 || n > CGKS_MLP_NOALLOC_MAX_ROWS) return n > CGKS_MLP_NOALLOC_MAX_ROWS ? CGKS_ELIMIT : CGKS_EINVAL;
    if (n == 0) return CGKS_OK;
    if (!X || !Y) return CGKS_EINVAL;
    __bf16* ws = nullptr;
    int rc = scratch_address(&ws);
    if (rc) return rc;
    __bf16* H0 = ws + NOALLOC_H0;
    __bf16* Hs[2] = {ws + NOALLOC_HA, ws + NOALLOC_HB};
    hipStream_t st = m->stream;
    /* the same kernels and arithmetic as cgks_mlp_forward; hidden layers
     * alternate between the two halves, the last layer writes Y directly */
    k_pack_input<<<nb((long)n * 32, 256), 256, 0, st>>>(X, H0, n);
    for (int l = 0; l < NL; ++l) {
        const __bf16* in = l == 0 ? H0 : Hs[(l - 1) & 1];
        if (l < NL - 1)
            gemm<EPI_BIAS_SILU_NOZ>(st, n, DOUT[l], KPAD[l], in, KPAD[l], 1, m->Wb[l], 1, KPAD[l], nullptr, 0,
                                    Hs[l & 1], KPAD[l + 1], m->P[l][1], nullptr, 0);
        else
            gemm<EPI_BIAS>(st, n, DOUT[l], KPAD[l], in, KPAD[l], 1, m->Wb[l], 1, KPAD[l], Y, 4, nullptr, 0,
                           m->P[l][1], nullptr, 0);
    }
    if (hipGetLastError() != hipSuccess) return CGKS_EDEVICE;
    return hipStreamSynchronize(st) == hipSuccess ? CGKS_OK : CGKS_EDEVICE;
}

int cgks_mlp_grads(cgks_mlp* m, const float* X, const float* Y, int n, float* grads_out, float* loss) {
    if (!m || !X || !Y || n <= 0) return CGKS_EINVAL;
    int rc = ensure_ws(m, n);
    if (rc) return rc;
    forward(m, X, n);
    backward(m, Y, n);
    if (hipStreamSynchronize(m->stream) != hipSuccess) return CGKS_EDEVICE;
    if (loss && hipMemcpy(loss, m->dloss, 4, hipMemcpyDeviceToHost) != hipSuccess) return CGKS_EDEVICE;
    if (grads_out) {
        size_t o = 0;
        for (int l = 0; l < NL; ++l) {
            std::vector<float> G(wcount(l));
            if (hipMemcpy(G.data(), m->Gr[l][0], G.size() * 4, hipMemcpyDeviceToHost) != hipSuccess) return CGKS_EDEVICE;
            for (int r = 0; r < DOUT[l]; ++r)
                for (int k = 0; k < DIN[l]; ++k) grads_out[o++] = G[(size_t)r * KPAD[l] + k];
            if (hipMemcpy(grads_out + o, m->Gr[l][1], DOUT[l] * 4, hipMemcpyDeviceToHost) != hipSuccess)
                return CGKS_EDEVICE;
            o += DOUT[l];
        }
    }
    return CGKS_OK;
}

int cgks_mlp_train_step(cgks_mlp* m, const float* X, const float* Y, int n, float lr, float* loss) {
    if (!m || !X || !Y || n <= 0 || !(lr > 0.0f)) return CGKS_EINVAL;
    int rc = ensure_ws(m, n);
    if (rc) return rc;
    forward(m, X, n);
    backward(m, Y, n);
    m->t += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - std::pow(b1, (float)m->t), c2 = 1.0f - std::pow(b2, (float)m->t);
    for (int l = 0; l < NL; ++l)
        for (int j = 0; j < 2; ++j) {
            const int cnt = j ? DOUT[l] : (int)wcount(l);
            k_adam<<<nb(cnt, 256), 256, 0, m->stream>>>(m->P[l][j], m->Gr[l][j], m->Mo[l][j], m->Vo[l][j],
                                                        j ? nullptr : m->Wb[l], cnt, lr, b1, b2, 1e-8f, c1, c2);
        }
    if (loss) {
        if (hipMemcpyAsync(loss, m->dloss, 4, hipMemcpyDeviceToHost, m->stream) != hipSuccess) return CGKS_EDEVICE;
    }
    return hipStreamSynchronize(m->stream) == hipSuccess ? CGKS_OK : CGKS_EDEVICE;
}

}  // extern "C"

/* Initial state from the network: features per fine cell (Mach, log10 Re,
 * x, y, distance to the nearest wall-face centre), standardised with fmean /
 * fstd; outputs de-standardised with tmean / tstd; cells whose prediction is
 * non-physical or non-finite fall back to the free stream. */
/* Raw features of a 2-D context's fine cells into the device array X [n][5]
 * (stream-ordered on the context's stream, synchronised). */
static int cell_features(cgks_ctx* c, float* X) {
    using namespace cgks;
    const HLevel& H = c->hl[0];
    std::vector<double> wc;
    for (const HFace& f : H.faces)
        if (f.R < 0 && (f.tag == CGKS_TAG_SLIP || f.tag == CGKS_TAG_ISOTHERMAL || f.tag == CGKS_TAG_ADIABATIC)) {
            wc.push_back(f.xc[0]);
            wc.push_back(f.xc[1]);
        }
    double* dwc = nullptr;
    if (!wc.empty() && (hipMalloc((void**)&dwc, wc.size() * 8) != hipSuccess ||
                        hipMemcpy(dwc, wc.data(), wc.size() * 8, hipMemcpyHostToDevice) != hipSuccess)) {
        (void)hipFree(dwc);
        return fail(c, CGKS_EDEVICE, "wall-centre upload failed");
    }
    const double lre = c->p.reynolds > 0.0 ? std::log10(c->p.reynolds) : 0.0;
    k_features<<<nb(H.n, 256), 256, 0, c->stream>>>(c->fine.C, H.n, dwc, (int)wc.size() / 2, c->p.mach, lre, X);
    const bool ok = hipGetLastError() == hipSuccess && hipStreamSynchronize(c->stream) == hipSuccess;
    (void)hipFree(dwc);
    return ok ? CGKS_OK : fail(c, CGKS_EDEVICE, "feature kernel failed");
}

extern "C" int cgks_init_from_mlp(cgks_ctx* c, cgks_mlp* m, const float* fmean, const float* fstd,
                                  const float* tmean, const float* tstd, int* n_fallback) {
    using namespace cgks;
    if (!c || !m || !fmean || !fstd || !tmean || !tstd) return CGKS_EINVAL;
    if (!c->have_mesh) return fail(c, CGKS_EINVAL, "no mesh");
    if (c->dim != 2) return fail(c, CGKS_EINVAL, "the warm start is defined for 2-D meshes");
    for (int k = 0; k < 5; ++k)
        if (!(fstd[k] > 0.0f)) return fail(c, CGKS_EINVAL, "feature scales must be positive");
    const int n = c->hl[0].n;
    float *dX = nullptr, *dt = nullptr, *dms = nullptr, *drg = nullptr;
    double *du = nullptr, *dW = nullptr;
    int *dfb = nullptr, *door = nullptr;
    int rc = CGKS_OK;
    float ms[10], tt[8];
    for (int k = 0; k < 5; ++k) {
        ms[k] = fmean[k];
        ms[5 + k] = fstd[k];
    }
    for (int k = 0; k < 4; ++k) {
        tt[k] = tmean[k];
        tt[4 + k] = tstd[k];
    }
    if (hipMalloc((void**)&dX, (size_t)n * 5 * 4) != hipSuccess || hipMalloc((void**)&dt, 8 * 4) != hipSuccess ||
        hipMalloc((void**)&dms, 10 * 4) != hipSuccess || hipMalloc((void**)&drg, 10 * 4) != hipSuccess ||
        hipMalloc((void**)&du, 3 * 8) != hipSuccess || hipMalloc((void**)&dW, (size_t)n * 4 * 8) != hipSuccess ||
        hipMalloc((void**)&dfb, 4) != hipSuccess || hipMalloc((void**)&door, (size_t)n * 4) != hipSuccess)
        rc = fail(c, CGKS_EDEVICE, "device allocation failed");
    if (rc == CGKS_OK) rc = ensure_ws(m, n);
    if (rc == CGKS_OK) rc = cell_features(c, dX);
    int fb = 0;
    if (rc == CGKS_OK) {
        bool ok = hipMemcpy(dt, tt, 8 * 4, hipMemcpyHostToDevice) == hipSuccess &&
                  hipMemcpy(dms, ms, 10 * 4, hipMemcpyHostToDevice) == hipSuccess &&
                  hipMemcpy(drg, m->range, 10 * 4, hipMemcpyHostToDevice) == hipSuccess &&
                  hipMemcpy(du, c->kp.u_inf, 3 * 8, hipMemcpyHostToDevice) == hipSuccess &&
                  hipMemset(dfb, 0, 4) == hipSuccess;
        if (ok) {
            hipStream_t keep = m->stream;
            m->stream = c->stream;
            k_standardise<<<nb(n, 256), 256, 0, c->stream>>>(dX, n, dms, m->have_range ? drg : nullptr, door);
            forward(m, dX, n);
            k_mlp_state<2><<<nb(n, 256), 256, 0, c->stream>>>(m->out, dt, c->p.mach, c->p.gamma, du, dW, n, dfb, door);
            m->stream = keep;
            ok = hipMemcpyAsync(&fb, dfb, 4, hipMemcpyDeviceToHost, c->stream) == hipSuccess &&
                 hipStreamSynchronize(c->stream) == hipSuccess;
        }
        rc = ok ? cgks_set_state(c, dW, nullptr, nullptr, CGKS_DEVICE) : fail(c, CGKS_EDEVICE, "warm start failed");
    }
    if (n_fallback) *n_fallback = fb;
    (void)hipFree(dX);
    (void)hipFree(dt);
    (void)hipFree(dms);
    (void)hipFree(drg);
    (void)hipFree(du);
    (void)hipFree(dW);
    (void)hipFree(dfb);
    (void)hipFree(door);
    return rc;
}

extern "C" int cgks_mlp_set_range(cgks_mlp* m, const float* lo, const float* hi) {
    if (!m) return CGKS_EINVAL;
    if (!lo || !hi) {
        m->have_range = false;
        return CGKS_OK;
    }
    for (int k = 0; k < 5; ++k)
        if (!(lo[k] <= hi[k])) return CGKS_EINVAL;
    for (int k = 0; k < 5; ++k) {
        m->range[k] = lo[k];
        m->range[5 + k] = hi[k];
    }
    m->have_range = true;
    return CGKS_OK;
}

extern "C" int cgks_mlp_features(cgks_ctx* c, float* X, int mem) {
    using namespace cgks;
    if (!c || !X || (mem != CGKS_HOST && mem != CGKS_DEVICE)) return CGKS_EINVAL;
    if (!c->have_mesh) return fail(c, CGKS_EINVAL, "no mesh");
    if (c->dim != 2) return fail(c, CGKS_EINVAL, "the warm start is defined for 2-D meshes");
    const int n = c->hl[0].n;
    if (mem == CGKS_DEVICE) return cell_features(c, X);
    float* dX = nullptr;
    if (hipMalloc((void**)&dX, (size_t)n * 5 * 4) != hipSuccess) return fail(c, CGKS_EDEVICE, "device allocation failed");
    int rc = cell_features(c, dX);
    if (rc == CGKS_OK && hipMemcpy(X, dX, (size_t)n * 5 * 4, hipMemcpyDeviceToHost) != hipSuccess)
        rc = fail(c, CGKS_EDEVICE, "copy of the features failed");
    (void)hipFree(dX);
    return rc;
}
