// Pricing surrogate of libamfrw: a fully connected network (SiLU hidden layers, BF16 weights and
// activations, FP32 accumulation on gfx950 MFMA) trained on prices produced by the solver, with a
// second output that estimates the network's own error and drives the fallback to the solver.
//
// Every matrix product is the same "NT" contraction C[M,N] = A[M,K] B[N,K]^T with both operands
// row-major in the contracted index, so 8 consecutive BF16 values feed one lane of
// v_mfma_f32_16x16x32_bf16:
//   forward   Z  = X  W^T + b          A = X   [B,K],  B = W  [N,K]
//   backward  dX = dZ W                A = dZ  [B,N],  B = W^T [K,N]
//   weights   dW = dZ^T X              A = dZ^T[N,B],  B = X^T [K,B]
// so the forward pass also stores activations transposed and the backward pass stores dZ^T.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "amfrw.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int TILE = 16;      // MFMA output tile 16 x 16
constexpr int KSTEP = 32;     // contraction per MFMA
constexpr int OUT_PAD = 32;   // output layer rows (price, error estimate) padded to a K step
constexpr int MAX_LAYERS = 8;

thread_local std::string g_mlp_err;

amf_status mfail(amf_status s, const std::string& m)
{
    g_mlp_err = m;
    return s;
}

__device__ __forceinline__ float bf2f(__bf16 x) { return (float)x; }
__device__ __forceinline__ __bf16 f2bf(float x) { return (__bf16)x; }   // round to nearest even

__device__ __forceinline__ float sigmoidf_(float z) { return 1.0f / (1.0f + __expf(-z)); }

enum GemmEpi : int {
    E_BIAS_SILU = 0,   // Z = C + b (FP32 store), A = silu(Z) -> BF16 row-major and transposed
    E_BIAS = 1,        // Y = C + b (FP32 store)
    E_DSILU = 2,       // dZ = C * silu'(Zprev) -> BF16 row-major and transposed
    E_STORE = 3        // C (FP32 store): weight gradients
};

struct GemmArgs {
    const __bf16* A;   // [M, K] row-major
    const __bf16* B;   // [N, K] row-major
    int M, N, K;
    const float* bias; // [N] (E_BIAS*)
    float* Cf;         // FP32 output [M, N] (Z, Y or dW)
    const float* Zin;  // E_DSILU: pre-activation [M, N]
    __bf16* Ob;        // BF16 output [M, N]
    __bf16* ObT;       // BF16 transposed output [N, ldT]
    int ldT;           // row stride of ObT (the padded batch)
};

// One wavefront per 16 x 16 tile of C; 4 wavefronts per block.
template <int EPI>
__global__ __launch_bounds__(256) void k_gemm_nt(GemmArgs g)
{
    const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int tn = g.N / TILE;
    const int tm_idx = wave / tn, tn_idx = wave % tn;
    if (tm_idx * TILE >= g.M) return;
    const int m0 = tm_idx * TILE, n0 = tn_idx * TILE;
    const int r = lane & 15, kb = lane >> 4;      // operand row, k-block of 8
    const __bf16* pa = g.A + (size_t)(m0 + r) * g.K + kb * 8;
    const __bf16* pb = g.B + (size_t)(n0 + r) * g.K + kb * 8;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int k = 0; k < g.K; k += KSTEP) {
        const bf16x8 a = *(const bf16x8*)(pa + k);
        const bf16x8 b = *(const bf16x8*)(pb + k);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
    }
    // lane holds C[m0 + 4*(lane/16) + i][n0 + lane%16], i = 0..3
    const int n = n0 + (lane & 15);
    const int mb = m0 + 4 * (lane >> 4);
    float v[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = acc[i];
    if constexpr (EPI == E_BIAS_SILU || EPI == E_BIAS) {
        const float bn = g.bias[n];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            v[i] += bn;
            g.Cf[(size_t)(mb + i) * g.N + n] = v[i];
        }
        if constexpr (EPI == E_BIAS_SILU) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const __bf16 a = f2bf(v[i] * sigmoidf_(v[i]));
                g.Ob[(size_t)(mb + i) * g.N + n] = a;
                g.ObT[(size_t)n * g.ldT + mb + i] = a;
            }
        }
    } else if constexpr (EPI == E_DSILU) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float z = g.Zin[(size_t)(mb + i) * g.N + n];
            const float s = sigmoidf_(z);
            const __bf16 d = f2bf(v[i] * s * (1.0f + z * (1.0f - s)));
            g.Ob[(size_t)(mb + i) * g.N + n] = d;
            g.ObT[(size_t)n * g.ldT + mb + i] = d;
        }
    } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) g.Cf[(size_t)(mb + i) * g.N + n] = v[i];
    }
}

// Inputs: x_norm = (x - mean) / std, zero-padded to kin columns and to the padded batch; BF16,
// row-major and transposed.
__global__ void k_input(const float* x, int batch, int nin, int kin, int bpad, const float* mean,
                        const float* stdv, __bf16* X, __bf16* XT)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= bpad * kin) return;
    const int b = i / kin, c = i % kin;
    float v = 0.0f;
    if (b < batch && c < nin) v = (x[(size_t)b * nin + c] - mean[c]) / stdv[c];
    const __bf16 h = f2bf(v);
    X[i] = h;
    XT[(size_t)c * bpad + b] = h;
}

// Outputs.  Linear target: price = y0 s0 + m0, relative error estimate exp(y1) s0 / |price|.
// Logarithmic target (omean[8] != 0): price = exp(y0 s0 + m0), relative error estimate exp(y1) s0.
__global__ void k_output(const float* Y, int batch, int ldy, const float* omean, const float* ostd,
                         float* out)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    const bool lg = omean[8] != 0.0f;
    const float u = Y[(size_t)b * ldy + 0] * ostd[0] + omean[0];
    const float price = lg ? __expf(u) : u;
    const float e = __expf(Y[(size_t)b * ldy + 1]) * ostd[0];
    out[2 * b + 0] = price;
    out[2 * b + 1] = lg ? e : e / fmaxf(fabsf(price), 1e-30f);
}

// Inference (no activations kept for a backward pass): one workgroup of four wavefronts takes
// INF_ROWS requests through every layer.  The layer input sits in LDS as BF16 rows; each wavefront
// computes the 16 x 16 output tiles of its columns (tiles w, w + 4, ... of the layer) for all rows,
// with the weights read as MFMA B operands from global memory (they stay in L2: every workgroup
// reads the same ones); bias and SiLU are applied in the epilogue and the BF16 result goes to the
// other LDS buffer.  Rounding points and accumulation order equal those of the training forward
// pass (k_input, k_gemm_nt, k_output), so the outputs are the same.
constexpr int INF_ROWS = 64;                 // requests per workgroup (4 row tiles)
constexpr int INF_MAXW = 256;                // widest layer input or output
constexpr int INF_LD = INF_MAXW + 8;         // LDS row pitch (BF16 elements): rows 4 banks apart

struct InferLayer {
    const __bf16* W;   // [N, K] row-major
    const float* b;    // [N]
    int N, K;
};
struct InferArgs {
    const float* x;
    int batch, nin, kin, nl;
    const float* mean;
    const float* stdv;
    const float* omean;
    const float* ostd;
    float* out;        // [batch, 2]
    InferLayer L[MAX_LAYERS];
};

__global__ __launch_bounds__(256) void k_mlp_infer(InferArgs A)
{
    __shared__ __align__(16) __bf16 buf[2][INF_ROWS * INF_LD];
    __shared__ float yout[INF_ROWS][2];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int row0 = blockIdx.x * INF_ROWS;
    // inputs, normalised and zero-padded to kin columns (rows past the batch are zero)
    for (int i = tid; i < INF_ROWS * A.kin; i += 256) {
        const int r = i / A.kin, c = i % A.kin, b = row0 + r;
        float v = 0.0f;
        if (b < A.batch && c < A.nin) v = (A.x[(size_t)b * A.nin + c] - A.mean[c]) / A.stdv[c];
        buf[0][r * INF_LD + c] = f2bf(v);
    }
    __syncthreads();
    const int r = lane & 15, kb = lane >> 4;
    for (int l = 0; l < A.nl; ++l) {
        const InferLayer Ly = A.L[l];
        const __bf16* in = buf[l & 1];
        __bf16* outb = buf[(l + 1) & 1];
        const bool last = l == A.nl - 1;
        const int tn = Ly.N / TILE;
        for (int ct0 = wave; ct0 < tn; ct0 += 16) {           // up to four column tiles per pass
            f32x4 acc[4][4];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
            for (int k = 0; k < Ly.K; k += KSTEP) {
                bf16x8 a[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) a[i] = *(const bf16x8*)(in + (i * TILE + r) * INF_LD + k + kb * 8);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int ct = ct0 + 4 * j;
                    if (ct < tn) {
                        const bf16x8 bv = *(const bf16x8*)(Ly.W + (size_t)(ct * TILE + r) * Ly.K + k + kb * 8);
#pragma unroll
                        for (int i = 0; i < 4; ++i) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], bv, acc[i][j], 0, 0, 0);
                    }
                }
            }
            // lane holds C[i*16 + 4*(lane/16) + e][ct*16 + lane%16], e = 0..3
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int ct = ct0 + 4 * j;
                if (ct >= tn) continue;
                const int n = ct * TILE + (lane & 15);
                const float bn = Ly.b[n];
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int m = i * TILE + 4 * (lane >> 4) + e;
                        const float v = acc[i][j][e] + bn;
                        if (!last) outb[m * INF_LD + n] = f2bf(v * sigmoidf_(v));
                        else if (n < 2) yout[m][n] = v;
                    }
            }
        }
        __syncthreads();
    }
    // outputs as k_output
    if (tid < INF_ROWS && row0 + tid < A.batch) {
        const int b = row0 + tid;
        const bool lg = A.omean[8] != 0.0f;
        const float u = yout[tid][0] * A.ostd[0] + A.omean[0];
        const float price = lg ? __expf(u) : u;
        const float e = __expf(yout[tid][1]) * A.ostd[0];
        A.out[2 * b + 0] = price;
        A.out[2 * b + 1] = lg ? e : e / fmaxf(fabsf(price), 1e-30f);
    }
}

// Router of the price_or_fallback call: request b is served by the network when its features lie in
// the training box [lo, hi], its price p is finite and its calibrated error estimate e = calib est
// satisfies e <= tol or e |p| <= abs_floor; used[b] = 1 routes it to the solver.
__global__ void k_route(const float* out, const float* x, int batch, int nin, const float* box, float calib,
                        float tol, float abs_floor, double* prices, int32_t* used)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    bool inside = true;
    for (int c = 0; c < nin; ++c) {
        const float v = x[(size_t)b * nin + c];
        inside = inside && v >= box[c] && v <= box[32 + c];
    }
    const float p = out[2 * b + 0];
    const float e = calib * out[2 * b + 1];
    const bool finite = isfinite(p) && isfinite(e);
    const bool ok = inside && finite && (e <= tol || e * fabsf(p) <= abs_floor);
    prices[b] = (double)p;
    used[b] = ok ? 0 : 1;
}

// Loss and output gradient.  t = (target - m0)/s0, r = y0 - t;
//   L = mean_b [ r^2 + w (y1 - log(|r| + eps))^2 ]   (the second term trains the error head on the
//   detached residual).  dY is written in BF16 row-major and transposed; padding rows/cols are 0.
__global__ void k_loss(const float* Y, const float* target, int batch, int bpad, int ldy,
                       const float* omean, const float* ostd, float wdet, __bf16* dY, __bf16* dYT,
                       float* row_loss)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= bpad) return;
    float g0 = 0.f, g1 = 0.f, l = 0.f;
    if (b < batch) {
        const float tv = omean[8] != 0.0f ? __logf(target[b]) : target[b];
        const float t = (tv - omean[0]) / ostd[0];
        const float y0 = Y[(size_t)b * ldy + 0], y1 = Y[(size_t)b * ldy + 1];
        const float rres = y0 - t;
        const float e = y1 - __logf(fabsf(rres) + 1e-6f);
        l = rres * rres + wdet * e * e;
        g0 = 2.0f * rres / (float)batch;
        g1 = 2.0f * wdet * e / (float)batch;
    }
    row_loss[b] = l;
    for (int c = 0; c < ldy; ++c) {
        const float gv = c == 0 ? g0 : (c == 1 ? g1 : 0.0f);
        const __bf16 h = f2bf(gv);
        dY[(size_t)b * ldy + c] = h;
        dYT[(size_t)c * bpad + b] = h;
    }
}

// Bias gradient: db[n] = sum_b dZ^T[n][b]; one block per n.  Also the loss sum (n = -1 row).
__global__ void k_rowsum_bf(const __bf16* A, int ld, int len, float* out)
{
    __shared__ float red[256];
    float s = 0.f;
    const __bf16* row = A + (size_t)blockIdx.x * ld;
    for (int i = threadIdx.x; i < len; i += blockDim.x) s += bf2f(row[i]);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

__global__ void k_sum_f(const float* a, int len, float* out)
{
    __shared__ float red[256];
    float s = 0.f;
    for (int i = threadIdx.x; i < len; i += blockDim.x) s += a[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

struct LayerDev {
    int N, K;            // padded output / input width
    int64_t w, b;        // offsets (floats) of W [N,K] and b [N] in the parameter vector
    int64_t wb, wtb;     // offsets (bf16 elements) of W and W^T in the BF16 weight buffer
};

// Adam on FP32 master weights; refreshes the BF16 copies W and W^T.  Padded rows/columns are kept
// at zero (masked gradient).
__global__ void k_adam(float* p, const float* grad, float* m, float* v, int64_t n, float lr, float b1,
                       float b2, float eps, float c1, float c2, const float* mask, __bf16* wbf,
                       const int64_t* bf_index, const int64_t* bft_index)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float g = grad[i] * mask[i];
    const float mi = b1 * m[i] + (1.f - b1) * g;
    const float vi = b2 * v[i] + (1.f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    const float w = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps) * mask[i];
    p[i] = w;
    if (bf_index[i] >= 0) {
        wbf[bf_index[i]] = f2bf(w);
        wbf[bft_index[i]] = f2bf(w);
    }
}

// Refresh the BF16 copies from the FP32 master weights.
__global__ void k_cast_params(const float* p, int64_t n, __bf16* wbf, const int64_t* bf_index,
                              const int64_t* bft_index)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || bf_index[i] < 0) return;
    wbf[bf_index[i]] = f2bf(p[i]);
    wbf[bft_index[i]] = f2bf(p[i]);
}

// dY (FP32 [batch, 2]) to BF16 [bp, OUT_PAD] and transposed, zero-padded.
__global__ void k_dy_from_f32(const float* dy, int batch, int bp, __bf16* D, __bf16* DT)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= bp) return;
    for (int c = 0; c < OUT_PAD; ++c) {
        const float v = (b < batch && c < 2) ? dy[2 * b + c] : 0.f;
        D[(size_t)b * OUT_PAD + c] = f2bf(v);
        DT[(size_t)c * bp + b] = f2bf(v);
    }
}

size_t a256(size_t x) { return (x + 255) / 256 * 256; }

}  // namespace

struct amf_mlp {
    int n_in = 0, width = 0, depth = 0, n_out = 0, max_batch = 0, bpad_max = 0;
    int nl = 0;                      // layers = depth + 1
    LayerDev L[MAX_LAYERS]{};
    int64_t n_params = 0, n_bf = 0;
    uint64_t seed = 0;
    std::vector<float> init_params, mask;
    std::vector<int64_t> bf_index, bft_index;
    // workspace offsets (bytes)
    size_t o_p = 0, o_g = 0, o_m = 0, o_v = 0, o_mask = 0, o_bfi = 0, o_bfti = 0, o_wbf = 0;
    size_t o_norm = 0, o_x = 0, o_xt = 0, o_z[MAX_LAYERS]{}, o_a[MAX_LAYERS]{}, o_at[MAX_LAYERS]{};
    size_t o_dy = 0, o_dyt = 0, o_dz = 0, o_dzt = 0, o_dzb = 0, o_dztb = 0, o_rl = 0, o_loss = 0;
    size_t o_route = 0, o_box = 0;   // router: network outputs [max_batch, 2]; box lo[32], hi[32]
    float calib = 1.0f;
    bool have_router = false;
    size_t ws_bytes = 0;
    char* ws = nullptr;
    int64_t t = 0;                   // Adam step
    int last_batch = 0, last_bpad = 0;
    bool have_forward = false;
    template <class T>
    T* at(size_t o) const { return (T*)(ws + o); }
};

namespace {

uint64_t splitmix(uint64_t& s)
{
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

int pad_to(int x, int m) { return (x + m - 1) / m * m; }

hipError_t gemm(int epi, const GemmArgs& g, hipStream_t s)
{
    const int tiles = (g.M / TILE) * (g.N / TILE);
    dim3 grid((tiles + 3) / 4), block(256);
    switch (epi) {
    case E_BIAS_SILU: hipLaunchKernelGGL(k_gemm_nt<E_BIAS_SILU>, grid, block, 0, s, g); break;
    case E_BIAS: hipLaunchKernelGGL(k_gemm_nt<E_BIAS>, grid, block, 0, s, g); break;
    case E_DSILU: hipLaunchKernelGGL(k_gemm_nt<E_DSILU>, grid, block, 0, s, g); break;
    default: hipLaunchKernelGGL(k_gemm_nt<E_STORE>, grid, block, 0, s, g); break;
    }
    return hipGetLastError();
}

amf_status hipchk(hipError_t e, const char* w)
{
    return e == hipSuccess ? AMF_OK : mfail(AMF_E_HIP, std::string(w) + ": " + hipGetErrorString(e));
}

// Forward pass for `batch` rows of raw features x (device FP32 [batch, n_in]).
amf_status forward(amf_mlp* N, const float* x, int batch, hipStream_t s)
{
    const int bp = pad_to(batch, KSTEP);
    const int kin = N->L[0].K;
    const float* norm = N->at<float>(N->o_norm);
    const int tot = bp * kin;
    hipLaunchKernelGGL(k_input, dim3((tot + 255) / 256), dim3(256), 0, s, x, batch, N->n_in, kin, bp,
                       norm, norm + 16, N->at<__bf16>(N->o_x), N->at<__bf16>(N->o_xt));
    amf_status st = hipchk(hipGetLastError(), "input");
    if (st) return st;
    const __bf16* wbf = N->at<__bf16>(N->o_wbf);
    const float* p = N->at<float>(N->o_p);
    const __bf16* in = N->at<__bf16>(N->o_x);
    for (int l = 0; l < N->nl; ++l) {
        const LayerDev& Ld = N->L[l];
        GemmArgs g{};
        g.A = in;
        g.B = wbf + Ld.wb;
        g.M = bp;
        g.N = Ld.N;
        g.K = Ld.K;
        g.bias = p + Ld.b;
        g.Cf = N->at<float>(N->o_z[l]);
        g.Ob = N->at<__bf16>(N->o_a[l]);
        g.ObT = N->at<__bf16>(N->o_at[l]);
        g.ldT = bp;
        if ((st = hipchk(gemm(l + 1 < N->nl ? E_BIAS_SILU : E_BIAS, g, s), "gemm fwd"))) return st;
        in = g.Ob;
    }
    N->last_batch = batch;
    N->last_bpad = bp;
    N->have_forward = true;
    return AMF_OK;
}

// Backward pass from dY (BF16 [bp, N_out] and transposed, already in the workspace) into the
// gradient vector (FP32, same layout as the parameters).
amf_status backward(amf_mlp* N, hipStream_t s)
{
    const int bp = N->last_bpad;
    amf_status st;
    const __bf16* wbf = N->at<__bf16>(N->o_wbf);
    float* grad = N->at<float>(N->o_g);
    const __bf16* dz = N->at<__bf16>(N->o_dy);
    const __bf16* dzt = N->at<__bf16>(N->o_dyt);
    for (int l = N->nl - 1; l >= 0; --l) {
        const LayerDev& Ld = N->L[l];
        // dW = dZ^T X (contraction over the batch)
        GemmArgs gw{};
        gw.A = dzt;
        gw.B = l == 0 ? N->at<__bf16>(N->o_xt) : N->at<__bf16>(N->o_at[l - 1]);
        gw.M = Ld.N;
        gw.N = Ld.K;
        gw.K = bp;
        gw.Cf = grad + Ld.w;
        if ((st = hipchk(gemm(E_STORE, gw, s), "gemm dW"))) return st;
        hipLaunchKernelGGL(k_rowsum_bf, dim3(Ld.N), dim3(256), 0, s, dzt, bp, bp, grad + Ld.b);
        if ((st = hipchk(hipGetLastError(), "db"))) return st;
        if (l == 0) break;
        // dX = dZ W, then through SiLU' of the previous layer
        GemmArgs gx{};
        gx.A = dz;
        gx.B = wbf + Ld.wtb;
        gx.M = bp;
        gx.N = Ld.K;
        gx.K = Ld.N;
        gx.Zin = N->at<float>(N->o_z[l - 1]);
        const bool flip = (l % 2) == 0;
        gx.Ob = N->at<__bf16>(flip ? N->o_dzb : N->o_dz);
        gx.ObT = N->at<__bf16>(flip ? N->o_dztb : N->o_dzt);
        gx.ldT = bp;
        if ((st = hipchk(gemm(E_DSILU, gx, s), "gemm dX"))) return st;
        dz = gx.Ob;
        dzt = gx.ObT;
    }
    return AMF_OK;
}

}  // namespace

extern "C" {

const char* amf_mlp_last_error(void) { return g_mlp_err.c_str(); }

amf_status amf_mlp_create(int32_t n_in, int32_t width, int32_t depth, int32_t n_out, int32_t max_batch,
                          uint64_t seed, amf_mlp** out)
{
    if (!out) return mfail(AMF_E_INVALID, "null output");
    *out = nullptr;
    if (n_in < 1 || n_in > 32) return mfail(AMF_E_INVALID, "n_in must lie in [1, 32]");
    if (n_out != 2) return mfail(AMF_E_UNSUPPORTED, "n_out must be 2 (price, error estimate)");
    if (width < 16 || width > 1024 || width % 32) return mfail(AMF_E_INVALID, "width must be a multiple of 32 in [32, 1024]");
    if (depth < 1 || depth > MAX_LAYERS - 1) return mfail(AMF_E_INVALID, "depth must lie in [1, 7]");
    if (max_batch < 1 || max_batch > (1 << 20)) return mfail(AMF_E_INVALID, "max_batch must lie in [1, 2^20]");
    amf_mlp* N = new (std::nothrow) amf_mlp();
    if (!N) return mfail(AMF_E_NOMEM, "out of host memory");
    N->n_in = n_in;
    N->width = width;
    N->depth = depth;
    N->n_out = n_out;
    N->max_batch = max_batch;
    N->bpad_max = pad_to(max_batch, KSTEP);
    N->seed = seed;
    N->nl = depth + 1;
    // layers: K padded to KSTEP at the input, N padded to OUT_PAD at the output
    int64_t po = 0, bo = 0;
    for (int l = 0; l < N->nl; ++l) {
        LayerDev& Ld = N->L[l];
        Ld.K = l == 0 ? KSTEP : width;
        Ld.N = l + 1 < N->nl ? width : OUT_PAD;
        Ld.w = po;
        po += (int64_t)Ld.N * Ld.K;
        Ld.b = po;
        po += Ld.N;
        Ld.wb = bo;
        bo += (int64_t)Ld.N * Ld.K;
        Ld.wtb = bo;
        bo += (int64_t)Ld.N * Ld.K;
    }
    N->n_params = po;
    N->n_bf = bo;
    // seeded uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases, zero padding
    N->init_params.assign(po, 0.f);
    N->mask.assign(po, 0.f);
    N->bf_index.assign(po, -1);
    N->bft_index.assign(po, -1);
    uint64_t st = seed;
    for (int l = 0; l < N->nl; ++l) {
        const LayerDev& Ld = N->L[l];
        const int kin = l == 0 ? n_in : width;
        const int nout = l + 1 < N->nl ? width : n_out;
        const float bound = 1.0f / std::sqrt((float)kin);
        for (int r = 0; r < Ld.N; ++r)
            for (int c = 0; c < Ld.K; ++c) {
                const int64_t i = Ld.w + (int64_t)r * Ld.K + c;
                N->bf_index[i] = Ld.wb + (int64_t)r * Ld.K + c;
                N->bft_index[i] = Ld.wtb + (int64_t)c * Ld.N + r;
                if (r < nout && c < kin) {
                    const double u = (double)(splitmix(st) >> 11) * (1.0 / 9007199254740992.0);
                    N->init_params[i] = (float)((2.0 * u - 1.0) * bound);
                    N->mask[i] = 1.f;
                }
            }
        for (int r = 0; r < nout; ++r) N->mask[Ld.b + r] = 1.f;
    }
    // workspace layout
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = a256(o + bytes);
        return at;
    };
    const size_t P = (size_t)po;
    const int bp = N->bpad_max;
    N->o_p = take(P * 4);
    N->o_g = take(P * 4);
    N->o_m = take(P * 4);
    N->o_v = take(P * 4);
    N->o_mask = take(P * 4);
    N->o_bfi = take(P * 8);
    N->o_bfti = take(P * 8);
    N->o_wbf = take((size_t)bo * 2);
    N->o_norm = take(64 * 4);
    N->o_x = take((size_t)bp * KSTEP * 2);
    N->o_xt = take((size_t)bp * KSTEP * 2);
    for (int l = 0; l < N->nl; ++l) {
        const int nw = N->L[l].N;
        N->o_z[l] = take((size_t)bp * nw * 4);
        N->o_a[l] = take((size_t)bp * nw * 2);
        N->o_at[l] = take((size_t)bp * nw * 2);
    }
    N->o_dy = take((size_t)bp * OUT_PAD * 2);
    N->o_dyt = take((size_t)bp * OUT_PAD * 2);
    N->o_dz = take((size_t)bp * width * 2);
    N->o_dzt = take((size_t)bp * width * 2);
    N->o_dzb = take((size_t)bp * width * 2);
    N->o_dztb = take((size_t)bp * width * 2);
    N->o_rl = take((size_t)bp * 4);
    N->o_loss = take(16);
    N->o_route = take((size_t)max_batch * 2 * 4);
    N->o_box = take(64 * 4);
    N->ws_bytes = o;
    *out = N;
    return AMF_OK;
}

amf_status amf_mlp_info_get(const amf_mlp* N, amf_mlp_info* out)
{
    if (!N || !out) return mfail(AMF_E_INVALID, "null argument");
    out->n_params = N->n_params;
    out->workspace_bytes = N->ws_bytes;
    out->n_in = N->n_in;
    out->width = N->width;
    out->depth = N->depth;
    out->n_out = N->n_out;
    out->max_batch = N->max_batch;
    out->layers = N->nl;
    for (int l = 0; l < N->nl; ++l) {
        out->layer_rows[l] = N->L[l].N;
        out->layer_cols[l] = N->L[l].K;
        out->layer_w_offset[l] = N->L[l].w;
        out->layer_b_offset[l] = N->L[l].b;
    }
    return AMF_OK;
}

amf_status amf_mlp_bind(amf_mlp* N, void* d_ws, uint64_t bytes, void* stream)
{
    if (!N || !d_ws) return mfail(AMF_E_INVALID, "null argument");
    if (bytes < N->ws_bytes) return mfail(AMF_E_INVALID, "workspace too small");
    if (((uintptr_t)d_ws & 255u) != 0) return mfail(AMF_E_INVALID, "workspace must be 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    N->ws = (char*)d_ws;
    N->t = 0;
    N->have_forward = false;
    const size_t P = (size_t)N->n_params;
    std::vector<float> zeros(P, 0.f);
    float normd[64];
    for (int i = 0; i < 64; ++i) normd[i] = (i < 16 || (i >= 32 && i < 48)) ? 0.f : 1.f;   // means 0, stds 1
    amf_status st;
    if ((st = hipchk(hipMemcpyAsync(N->ws + N->o_p, N->init_params.data(), P * 4, hipMemcpyHostToDevice, s), "upload"))) return st;
    if ((st = hipchk(hipMemcpyAsync(N->ws + N->o_m, zeros.data(), P * 4, hipMemcpyHostToDevice, s), "upload"))) return st;
    if ((st = hipchk(hipMemcpyAsync(N->ws + N->o_v, zeros.data(), P * 4, hipMemcpyHostToDevice, s), "upload"))) return st;
    if ((st = hipchk(hipMemcpyAsync(N->ws + N->o_g, zeros.data(), P * 4, hipMemcpyHostToDevice, s), "upload"))) return st;
    if ((st = hipchk(hipMemcpyAsync(N->ws + N->o_mask, N->mask.data(), P * 4, hipMemcpyHostToDevice, s), "upload"))) return st;
    if ((st = hipchk(hipMemcpyAsync(N->ws + N->o_bfi, N->bf_index.data(), P * 8, hipMemcpyHostToDevice, s), "upload"))) return st;
    if ((st = hipchk(hipMemcpyAsync(N->ws + N->o_bfti, N->bft_index.data(), P * 8, hipMemcpyHostToDevice, s), "upload"))) return st;
    if ((st = hipchk(hipMemcpyAsync(N->ws + N->o_norm, normd, sizeof(normd), hipMemcpyHostToDevice, s), "upload"))) return st;
    hipLaunchKernelGGL(k_cast_params, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, N->at<float>(N->o_p),
                       (int64_t)P, N->at<__bf16>(N->o_wbf), N->at<int64_t>(N->o_bfi), N->at<int64_t>(N->o_bfti));
    if ((st = hipchk(hipGetLastError(), "cast"))) return st;
    return hipchk(hipStreamSynchronize(s), "hipStreamSynchronize");
}

amf_status amf_mlp_set_normalization(amf_mlp* N, const float* in_mean, const float* in_std,
                                     const float* out_mean, const float* out_std, int32_t out_log,
                                     void* stream)
{
    if (out_log != 0 && out_log != 1) return mfail(AMF_E_INVALID, "out_log must be 0 or 1");
    if (!N || !N->ws || !in_mean || !in_std || !out_mean || !out_std) return mfail(AMF_E_INVALID, "null argument");
    float normd[64];
    for (int i = 0; i < 16; ++i) {
        normd[i] = i < N->n_in ? in_mean[i] : 0.f;
        normd[16 + i] = i < N->n_in ? in_std[i] : 1.f;
        normd[32 + i] = i < 1 ? out_mean[0] : (i == 8 ? (float)out_log : 0.f);
        normd[48 + i] = i < 1 ? out_std[0] : 1.f;
    }
    for (int i = 0; i < N->n_in; ++i)
        if (!(in_std[i] > 0.f)) return mfail(AMF_E_INVALID, "in_std must be > 0");
    if (!(out_std[0] > 0.f)) return mfail(AMF_E_INVALID, "out_std must be > 0");
    hipStream_t s = (hipStream_t)stream;
    amf_status st = hipchk(hipMemcpyAsync(N->ws + N->o_norm, normd, sizeof(normd), hipMemcpyHostToDevice, s), "upload");
    if (st) return st;
    return hipchk(hipStreamSynchronize(s), "hipStreamSynchronize");
}

amf_status amf_mlp_params(amf_mlp* N, float* d_params, int32_t direction, void* stream)
{
    if (!N || !N->ws || !d_params) return mfail(AMF_E_INVALID, "null argument");
    hipStream_t s = (hipStream_t)stream;
    const size_t P = (size_t)N->n_params;
    if (direction == 0)
        return hipchk(hipMemcpyAsync(d_params, N->ws + N->o_p, P * 4, hipMemcpyDeviceToDevice, s), "copy");
    amf_status st = hipchk(hipMemcpyAsync(N->ws + N->o_p, d_params, P * 4, hipMemcpyDeviceToDevice, s), "copy");
    if (st) return st;
    hipLaunchKernelGGL(k_cast_params, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, N->at<float>(N->o_p),
                       (int64_t)P, N->at<__bf16>(N->o_wbf), N->at<int64_t>(N->o_bfi), N->at<int64_t>(N->o_bfti));
    return hipchk(hipGetLastError(), "cast");
}

amf_status amf_mlp_grads(amf_mlp* N, float* d_grads, void* stream)
{
    if (!N || !N->ws || !d_grads) return mfail(AMF_E_INVALID, "null argument");
    return hipchk(hipMemcpyAsync(d_grads, N->ws + N->o_g, (size_t)N->n_params * 4, hipMemcpyDeviceToDevice,
                                 (hipStream_t)stream), "copy");
}

amf_status amf_mlp_forward(amf_mlp* N, const float* d_x, int32_t batch, float* d_out, void* stream)
{
    if (!N || !N->ws || !d_x || !d_out) return mfail(AMF_E_INVALID, "null argument");
    if (batch < 1 || batch > N->max_batch) return mfail(AMF_E_INVALID, "batch out of range");
    hipStream_t s = (hipStream_t)stream;
    amf_status st = forward(N, d_x, batch, s);
    if (st) return st;
    const LayerDev& Lo = N->L[N->nl - 1];
    const float* norm = N->at<float>(N->o_norm);
    hipLaunchKernelGGL(k_output, dim3((batch + 255) / 256), dim3(256), 0, s, N->at<float>(N->o_z[N->nl - 1]),
                       batch, Lo.N, norm + 32, norm + 48, d_out);
    return hipchk(hipGetLastError(), "output");
}

amf_status amf_mlp_infer(amf_mlp* N, const float* d_x, int32_t batch, float* d_out, void* stream)
{
    if (!N || !N->ws || !d_x || !d_out) return mfail(AMF_E_INVALID, "null argument");
    if (batch < 1) return mfail(AMF_E_INVALID, "batch must be >= 1");
    hipStream_t s = (hipStream_t)stream;
    bool fits = N->nl <= MAX_LAYERS && N->L[0].K <= INF_MAXW && N->L[N->nl - 1].N >= 2;
    for (int l = 0; l < N->nl; ++l) fits = fits && N->L[l].N <= INF_MAXW && N->L[l].K <= INF_MAXW;
    if (!fits) {                                  // wider networks: the training forward pass, in chunks
        for (int c0 = 0; c0 < batch; c0 += N->max_batch) {
            const int b = std::min(N->max_batch, batch - c0);
            amf_status st = amf_mlp_forward(N, d_x + (size_t)c0 * N->n_in, b, d_out + 2 * (size_t)c0, stream);
            if (st) return st;
        }
        return AMF_OK;
    }
    InferArgs a{};
    a.x = d_x;
    a.batch = batch;
    a.nin = N->n_in;
    a.kin = N->L[0].K;
    a.nl = N->nl;
    const float* norm = N->at<float>(N->o_norm);
    a.mean = norm;
    a.stdv = norm + 16;
    a.omean = norm + 32;
    a.ostd = norm + 48;
    a.out = d_out;
    const __bf16* wbf = N->at<__bf16>(N->o_wbf);
    const float* p = N->at<float>(N->o_p);
    for (int l = 0; l < N->nl; ++l) a.L[l] = InferLayer{wbf + N->L[l].wb, p + N->L[l].b, N->L[l].N, N->L[l].K};
    hipLaunchKernelGGL(k_mlp_infer, dim3((unsigned)((batch + INF_ROWS - 1) / INF_ROWS)), dim3(256), 0, s, a);
    return hipchk(hipGetLastError(), "infer");
}

amf_status amf_mlp_set_router(amf_mlp* N, const float* box_lo, const float* box_hi, float calib)
{
    if (!N || !N->ws || !box_lo || !box_hi) return mfail(AMF_E_INVALID, "null argument");
    if (!(calib > 0.0f) || !std::isfinite(calib)) return mfail(AMF_E_INVALID, "calib must be > 0");
    float box[64];
    for (int c = 0; c < 32; ++c) {
        box[c] = c < N->n_in ? box_lo[c] : 0.0f;
        box[32 + c] = c < N->n_in ? box_hi[c] : 0.0f;
        if (c < N->n_in && !(box_lo[c] <= box_hi[c])) return mfail(AMF_E_INVALID, "box_lo must be <= box_hi");
    }
    hipError_t e = hipMemcpy(N->ws + N->o_box, box, sizeof(box), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hipchk(e, "upload");
    N->calib = calib;
    N->have_router = true;
    return AMF_OK;
}

amf_status amf_mlp_backward(amf_mlp* N, const float* d_dy, int32_t batch, void* stream)
{
    if (!N || !N->ws || !d_dy) return mfail(AMF_E_INVALID, "null argument");
    if (!N->have_forward || batch != N->last_batch) return mfail(AMF_E_STATE, "backward needs the forward pass of the same batch");
    hipStream_t s = (hipStream_t)stream;
    // dY given in FP32 [batch, 2] (gradient w.r.t. the raw network outputs y0, y1)
    const int bp = N->last_bpad;
    hipLaunchKernelGGL(k_dy_from_f32, dim3((bp + 255) / 256), dim3(256), 0, s, d_dy, batch, bp,
                       N->at<__bf16>(N->o_dy), N->at<__bf16>(N->o_dyt));
    amf_status st = hipchk(hipGetLastError(), "dy");
    if (st) return st;
    return backward(N, s);
}

amf_status amf_mlp_train_step(amf_mlp* N, const float* d_x, const float* d_target, int32_t batch,
                              float lr, float err_weight, float* d_loss, void* stream)
{
    if (!N || !N->ws || !d_x || !d_target) return mfail(AMF_E_INVALID, "null argument");
    if (batch < 1 || batch > N->max_batch) return mfail(AMF_E_INVALID, "batch out of range");
    if (!(lr > 0.f) || !(err_weight >= 0.f)) return mfail(AMF_E_INVALID, "lr must be > 0, err_weight >= 0");
    hipStream_t s = (hipStream_t)stream;
    amf_status st = forward(N, d_x, batch, s);
    if (st) return st;
    const int bp = N->last_bpad;
    const LayerDev& Lo = N->L[N->nl - 1];
    const float* norm = N->at<float>(N->o_norm);
    hipLaunchKernelGGL(k_loss, dim3((bp + 255) / 256), dim3(256), 0, s, N->at<float>(N->o_z[N->nl - 1]), d_target,
                       batch, bp, Lo.N, norm + 32, norm + 48, err_weight, N->at<__bf16>(N->o_dy),
                       N->at<__bf16>(N->o_dyt), N->at<float>(N->o_rl));
    if ((st = hipchk(hipGetLastError(), "loss"))) return st;
    hipLaunchKernelGGL(k_sum_f, dim3(1), dim3(256), 0, s, N->at<float>(N->o_rl), bp, N->at<float>(N->o_loss));
    if ((st = hipchk(hipGetLastError(), "loss sum"))) return st;
    if (d_loss && (st = hipchk(hipMemcpyAsync(d_loss, N->ws + N->o_loss, 4, hipMemcpyDeviceToDevice, s), "copy"))) return st;
    if ((st = backward(N, s))) return st;
    N->t += 1;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - std::pow(b1, (float)N->t), c2 = 1.f - std::pow(b2, (float)N->t);
    const size_t P = (size_t)N->n_params;
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, N->at<float>(N->o_p),
                       N->at<float>(N->o_g), N->at<float>(N->o_m), N->at<float>(N->o_v), (int64_t)P, lr, b1, b2,
                       eps, c1, c2, N->at<float>(N->o_mask), N->at<__bf16>(N->o_wbf), N->at<int64_t>(N->o_bfi),
                       N->at<int64_t>(N->o_bfti));
    return hipchk(hipGetLastError(), "adam");
}

void amf_mlp_destroy(amf_mlp* N) { delete N; }

}  // extern "C"

namespace amf {

// Network prices and routing decisions for n requests (chunks of max_batch): d_prices[i] = the
// network's price, d_used[i] = 1 when request i must go to the solver.
amf_status mlp_route(amf_mlp* N, const float* d_x, int64_t n, float tol, float abs_floor, double* d_prices,
                     int32_t* d_used, hipStream_t s)
{
    if (!N || !N->ws || !d_x || !d_prices || !d_used) return mfail(AMF_E_INVALID, "null argument");
    if (!N->have_router) return mfail(AMF_E_STATE, "amf_mlp_set_router has not been called");
    if (!(tol >= 0.0f) || !(abs_floor >= 0.0f)) return mfail(AMF_E_INVALID, "tol and abs_floor must be >= 0");
    float* out = (float*)(N->ws + N->o_route);
    for (int64_t c0 = 0; c0 < n; c0 += N->max_batch) {
        const int b = (int)std::min<int64_t>(N->max_batch, n - c0);
        amf_status st = amf_mlp_infer(N, d_x + c0 * N->n_in, b, out, s);
        if (st) return st;
        hipLaunchKernelGGL(k_route, dim3((b + 255) / 256), dim3(256), 0, s, out, d_x + c0 * N->n_in, b, N->n_in,
                           (const float*)(N->ws + N->o_box), N->calib, tol, abs_floor, d_prices + c0, d_used + c0);
        if ((st = hipchk(hipGetLastError(), "route"))) return st;
    }
    return AMF_OK;
}

const char* mlp_error() { return g_mlp_err.c_str(); }

}  // namespace amf
