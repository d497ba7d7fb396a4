// mlp.hip -- gfx950 kernels of the learned per-block codec selector's network:
// 40 block features -> 64 -> 64 -> 16 class logits with ReLU, softmax
// cross-entropy plus an expected size-excess term, trained with Adam.
//
// Matrix products run on the matrix cores (v_mfma_f32_16x16x32_bf16, and
// v_mfma_f32_16x16x16_bf16 for a remaining 16 of K): bf16 operands, fp32
// accumulation.  Each workgroup of four waves takes 64 samples;
// wave w owns rows 16w..16w+15 in the forward pass and in the backward
// products through the layers, and the weight gradients are contractions
// over all 64 rows, one output tile row per wave.  Activations and
// gradients live in LDS as bf16; the bf16 weights are read from global
// memory (16 KB, cache resident) in the layouts the fragments want.
// Gradients of a batch are written per workgroup and summed in a fixed
// order by the reduce/Adam kernel, so a step is deterministic.
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "gc_mlp.h"

namespace gcmlp {

typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;

// fp32 -> bf16, round to nearest even (finite values)
__device__ __forceinline__ uint16_t to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ f32x4 mfma(s16x4 a, s16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma32(s16x8 a, s16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0,
                                                   0, 0);
}

// Fragments of a 16x16x16 product, lane l = 16q + i:
//   A (16 rows x 16 k): row r0 + i, k = k0 + 4q + j (j = 0..3)
//   B (16 k x 16 cols): col c0 + i, k = k0 + 4q + j
//   result: col c0 + i, rows r0 + 4q + e (e = 0..3)
// M[x][k] with k contiguous: one 8-byte load.
__device__ __forceinline__ s16x4 frag_kc(const uint16_t *M, int ld, int x0, int k0, int lane) {
    return *reinterpret_cast<const s16x4 *>(M + (x0 + (lane & 15)) * ld + k0 + 4 * (lane >> 4));
}
// Fragments of a 16x16x32 product, lane l = 16q + i: the same with
// k = k0 + 8q + j (j = 0..7).  M[x][k] with k contiguous: one 16-byte load
// (every row stride and k0 here is a multiple of 8 elements).
__device__ __forceinline__ s16x8 frag8_kc(const uint16_t *M, int ld, int x0, int k0, int lane) {
    return *reinterpret_cast<const s16x8 *>(M + (x0 + (lane & 15)) * ld + k0 + 8 * (lane >> 4));
}

// M[k][x] with x contiguous: eight 2-byte loads.
__device__ __forceinline__ s16x8 frag8_ks(const uint16_t *M, int ld, int x0, int k0, int lane) {
    const uint16_t *p = M + (k0 + 8 * (lane >> 4)) * ld + x0 + (lane & 15);
    s16x8 r;
#pragma unroll
    for (int j = 0; j < 8; j++) r[j] = (short)p[j * ld];
    return r;
}

__device__ __forceinline__ float sum16(float x) {
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) x += __shfl_xor(x, o);
    return x;
}
__device__ __forceinline__ float max16(float x) {
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) x = fmaxf(x, __shfl_xor(x, o));
    return x;
}
// sum over the four lane groups q (lanes i, i+16, i+32, i+48)
__device__ __forceinline__ float sum_q(float x) {
    x += __shfl_xor(x, 16);
    x += __shfl_xor(x, 32);
    return x;
}

struct __align__(16) NetSmem {
    uint16_t a0[kRows * kInPad];
    uint16_t a1[kRows * kHid];
    uint16_t a2[kRows * kHid];
    uint16_t g3[kRows * kOut];
    uint16_t d2[kRows * kHid];
    uint16_t d1[kRows * kHid];
    float bsum[4][2 * kHid + kOut];   // per wave: db1, db2, db3 column sums
    float lsum[4];
};
// The forward pass alone uses the activations, the leading members: its
// workgroups take that much LDS (22 KB against 51 KB), so that seven fit a CU.
constexpr size_t kFwdSmem = offsetof(NetSmem, g3);

// One dense layer for a wave's 16 rows: out = bf(relu(in W + b)).
template <int KT>
__device__ __forceinline__ void dense_relu(const uint16_t *in, int ldin, const uint16_t *wt, const float *bias,
                                           uint16_t *out, int r0, int lane) {
    const int i = lane & 15, q = lane >> 4;
#pragma unroll
    for (int nt = 0; nt < kHid / 16; nt++) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kt = 0; kt + 1 < KT; kt += 2)
            acc = mfma32(frag8_kc(in, ldin, r0, 16 * kt, lane), frag8_kc(wt, KT * 16, 16 * nt, 16 * kt, lane), acc);
        if constexpr (KT % 2)
            acc = mfma(frag_kc(in, ldin, r0, 16 * (KT - 1), lane), frag_kc(wt, KT * 16, 16 * nt, 16 * (KT - 1), lane), acc);
        const int col = 16 * nt + i;
        const float b = bias[col];
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const float z = acc[e] + b;
            out[(r0 + 4 * q + e) * kHid + col] = to_bf16(z > 0.f ? z : 0.f);
        }
    }
}

// TRAIN: gradient partials of the batch; otherwise logits and/or classes.
template <bool TRAIN>
__global__ __launch_bounds__(kThreads) void gc_mlp_kernel(Batch b, const float *theta, Packed w, float *partial,
                                                          float *logits, uint8_t *cls) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    NetSmem &sm = *reinterpret_cast<NetSmem *>(smem_raw);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = lane & 15, q = lane >> 4, r0 = 16 * wave;
    const size_t base = (size_t)blockIdx.x * kRows;

    // The workgroup's 64 x 48 inputs (40 features, then zero padding).  The
    // loads are unconditional, a missing row or a padding column reading the
    // workgroup's first feature, so that a thread's twelve are in flight
    // together.
    constexpr int kLoads = kRows * kInPad / kThreads;
    static_assert(kRows * kInPad % kThreads == 0, "whole loads per thread");
    size_t src[kLoads];
#pragma unroll
    for (int j = 0; j < kLoads; j++) {
        const int e = threadIdx.x + j * kThreads, r = e / kInPad, k = e - r * kInPad;
        const bool ok = k < kIn && base + r < b.count;
        src[j] = b.row0 + (ok ? base + r : base);   // base < count
    }
    if (b.index) {   // the sample rows first, all at once
        uint32_t ix[kLoads];
#pragma unroll
        for (int j = 0; j < kLoads; j++) ix[j] = b.index[src[j]];
#pragma unroll
        for (int j = 0; j < kLoads; j++) src[j] = ix[j];
    }
    float x[kLoads];
#pragma unroll
    for (int j = 0; j < kLoads; j++) {
        const int e = threadIdx.x + j * kThreads, r = e / kInPad, k = e - r * kInPad;
        x[j] = b.feat[src[j] * kIn + (k < kIn ? k : 0)];
    }
#pragma unroll
    for (int j = 0; j < kLoads; j++) {
        const int e = threadIdx.x + j * kThreads, r = e / kInPad, k = e - r * kInPad;
        sm.a0[e] = to_bf16(k < kIn && base + r < b.count ? x[j] : 0.f);
    }
    __syncthreads();
    dense_relu<3>(sm.a0, kInPad, w.w1t, theta + kOffB1, sm.a1, r0, lane);
    __syncthreads();
    dense_relu<4>(sm.a1, kHid, w.w2t, theta + kOffB2, sm.a2, r0, lane);
    __syncthreads();
    f32x4 z3 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kt = 0; kt < 4; kt += 2)
        z3 = mfma32(frag8_kc(sm.a2, kHid, r0, 16 * kt, lane), frag8_kc(w.w3t, kHid, 0, 16 * kt, lane), z3);
    const float b3 = theta[kOffB3 + i];

    if (!TRAIN) {
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const size_t row = base + r0 + 4 * q + e;
            const float z = z3[e] + b3;
            if (logits && row < b.count) logits[row * kOut + i] = z;
            // first class of the largest logit
            float bv = z;
            int bi = i;
#pragma unroll
            for (int o = 1; o < 16; o <<= 1) {
                const float ov = __shfl_xor(bv, o);
                const int oi = __shfl_xor(bi, o);
                if (ov > bv || (ov == bv && oi < bi)) {
                    bv = ov;
                    bi = oi;
                }
            }
            if (cls && i == 0 && row < b.count) cls[row] = (uint8_t)bi;
        }
        return;
    }

    // softmax, loss and G3 = (P - onehot + lam P (c - <P, c>)) / B
    const float inv_b = 1.0f / (float)b.count;
    float lacc = 0.f, db3 = 0.f;
    // labels and costs of the lane's four rows, loaded together (a missing
    // row reads the workgroup's first)
    float cst[4];
    uint32_t lab[4];
#pragma unroll
    for (int e = 0; e < 4; e++) {
        const int r = r0 + 4 * q + e;
        const size_t row = b.row0 + (base + r < b.count ? base + r : base);
        const size_t src = b.index ? (size_t)b.index[row] : row;
        cst[e] = b.cost ? b.cost[src * kOut + i] : 0.f;
        lab[e] = b.label[src];
    }
#pragma unroll
    for (int e = 0; e < 4; e++) {
        const int r = r0 + 4 * q + e;
        const bool valid = base + r < b.count;
        const float z = z3[e] + b3;
        const float mx = max16(z);
        const float ex = expf(z - mx);
        const float se = sum16(ex);
        const float p = ex / se;
        const float c = valid ? cst[e] : 0.f;
        const float ec = sum16(p * c);
        const bool hit = valid && (int)lab[e] == i;
        float g = 0.f;
        if (valid) {
            g = (p - (hit ? 1.f : 0.f) + b.lam * p * (c - ec)) * inv_b;
            lacc += (hit ? logf(se) + mx - z : 0.f) + b.lam * p * c;
        }
        db3 += g;
        sm.g3[r * kOut + i] = to_bf16(g);
    }
    db3 = sum_q(db3);
    if (q == 0) sm.bsum[wave][2 * kHid + i] = db3;
    for (int o = 1; o < 64; o <<= 1) lacc += __shfl_xor(lacc, o);
    if (lane == 0) sm.lsum[wave] = lacc * inv_b;
    __syncthreads();

    // dZ2 = bf(G3) bf(W3)^T masked by A2 > 0
#pragma unroll
    for (int nt = 0; nt < 4; nt++) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mfma(frag_kc(sm.g3, kOut, r0, 0, lane), frag_kc(w.w3, kOut, 16 * nt, 0, lane), acc);
        const int col = 16 * nt + i;
        float cs = 0.f;
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const int r = r0 + 4 * q + e;
            const float dz = sm.a2[r * kHid + col] ? acc[e] : 0.f;
            cs += dz;
            sm.d2[r * kHid + col] = to_bf16(dz);
        }
        cs = sum_q(cs);
        if (q == 0) sm.bsum[wave][kHid + col] = cs;
    }
    __syncthreads();
    // dZ1 = bf(dZ2) bf(W2)^T masked by A1 > 0
#pragma unroll
    for (int nt = 0; nt < 4; nt++) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kt = 0; kt < 4; kt += 2)
            acc = mfma32(frag8_kc(sm.d2, kHid, r0, 16 * kt, lane), frag8_kc(w.w2, kHid, 16 * nt, 16 * kt, lane), acc);
        const int col = 16 * nt + i;
        float cs = 0.f;
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const int r = r0 + 4 * q + e;
            const float dz = sm.a1[r * kHid + col] ? acc[e] : 0.f;
            cs += dz;
            sm.d1[r * kHid + col] = to_bf16(dz);
        }
        cs = sum_q(cs);
        if (q == 0) sm.bsum[wave][col] = cs;
    }
    __syncthreads();

    float *part = partial + (size_t)blockIdx.x * kPartialStride;
    // dW3 = A2^T bf(G3): hidden rows 16 wave.. of 64 x 16
    {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kt = 0; kt < 4; kt += 2)
            acc = mfma32(frag8_ks(sm.a2, kHid, r0, 16 * kt, lane), frag8_ks(sm.g3, kOut, 0, 16 * kt, lane), acc);
#pragma unroll
        for (int e = 0; e < 4; e++) part[kOffW3 + (r0 + 4 * q + e) * kOut + i] = acc[e];
    }
    // dW2 = A1^T bf(dZ2): input rows 16 wave.. of 64 x 64
#pragma unroll
    for (int ot = 0; ot < 4; ot++) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kt = 0; kt < 4; kt += 2)
            acc = mfma32(frag8_ks(sm.a1, kHid, r0, 16 * kt, lane), frag8_ks(sm.d2, kHid, 16 * ot, 16 * kt, lane), acc);
#pragma unroll
        for (int e = 0; e < 4; e++) part[kOffW2 + (r0 + 4 * q + e) * kHid + 16 * ot + i] = acc[e];
    }
    // dW1 = A0^T bf(dZ1): output columns 16 wave.. of 40 x 64
#pragma unroll
    for (int it = 0; it < 3; it++) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kt = 0; kt < 4; kt += 2)
            acc = mfma32(frag8_ks(sm.a0, kInPad, 16 * it, 16 * kt, lane), frag8_ks(sm.d1, kHid, r0, 16 * kt, lane), acc);
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const int in = 16 * it + 4 * q + e;
            if (in < kIn) part[kOffW1 + in * kHid + r0 + i] = acc[e];
        }
    }
    const int t = threadIdx.x;
    if (t < 2 * kHid + kOut) {
        const float s = sm.bsum[0][t] + sm.bsum[1][t] + sm.bsum[2][t] + sm.bsum[3][t];
        part[t < kHid ? kOffB1 + t : t < 2 * kHid ? kOffB2 + t - kHid : kOffB3 + t - 2 * kHid] = s;
    }
    if (t == 0) part[kParams] = sm.lsum[0] + sm.lsum[1] + sm.lsum[2] + sm.lsum[3];
}

// bf16 copies of parameter p
__device__ __forceinline__ void pack_one(int p, float val, const Packed &w) {
    const uint16_t h = to_bf16(val);
    if (p < kOffB1) {
        const int in = p / kHid, o = p - in * kHid;
        w.w1t[o * kInPad + in] = h;
    } else if (p >= kOffW2 && p < kOffB2) {
        const int x = p - kOffW2, in = x / kHid, o = x - in * kHid;
        w.w2t[o * kHid + in] = h;
        w.w2[in * kHid + o] = h;
    } else if (p >= kOffW3 && p < kOffB3) {
        const int x = p - kOffW3, h3 = x / kOut, c = x - h3 * kOut;
        w.w3t[c * kHid + h3] = h;
        w.w3[h3 * kOut + c] = h;
    }
}

__global__ __launch_bounds__(kThreads) void gc_mlp_reduce_adam_kernel(const float *partial, uint32_t nparts,
                                                                      float *grad, float *loss, float *theta,
                                                                      float *m, float *v, Packed w, int update,
                                                                      float lr, float beta1, float beta2, float eps,
                                                                      float c1, float c2) {
    const int p = blockIdx.x * kThreads + threadIdx.x;
    if (p > kParams) return;
    float g = 0.f;
    // in workgroup order; unrolled so that 16 loads are in flight at once
#pragma unroll 16
    for (uint32_t k = 0; k < nparts; k++) g += partial[(size_t)k * kPartialStride + p];
    if (p == kParams) {
        if (loss) *loss = g;
        return;
    }
    if (grad) grad[p] = g;
    if (update) {
        const float mm = beta1 * m[p] + (1.f - beta1) * g;
        const float vv = beta2 * v[p] + (1.f - beta2) * g * g;
        m[p] = mm;
        v[p] = vv;
        const float th = theta[p] - lr * (mm * c1) / (sqrtf(vv * c2) + eps);
        theta[p] = th;
        pack_one(p, th, w);
    }
}

__global__ __launch_bounds__(kThreads) void gc_mlp_pack_kernel(const float *theta, Packed w) {
    const int p = blockIdx.x * kThreads + threadIdx.x;
    if (p < kParams) pack_one(p, theta[p], w);
}

// ---- launchers -------------------------------------------------------------------

static unsigned groups(size_t rows) { return (unsigned)((rows + kRows - 1) / kRows); }

int launch_grad_partials(const Batch &b, const float *theta, const Packed &w, float *partial, hipStream_t s) {
    if (!b.count) return 0;
    hipLaunchKernelGGL(gc_mlp_kernel<true>, dim3(groups(b.count)), dim3(kThreads), sizeof(NetSmem), s, b, theta, w, partial,
                       (float *)nullptr, (uint8_t *)nullptr);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_reduce_adam(const float *partial, uint32_t nparts, float *grad, float *loss, float *theta, float *m,
                       float *v, const Packed &w, bool update, float lr, float beta1, float beta2, float eps,
                       float c1, float c2, hipStream_t s) {
    hipLaunchKernelGGL(gc_mlp_reduce_adam_kernel, dim3((kParams + kThreads) / kThreads), dim3(kThreads), 0, s,
                       partial, nparts, grad, loss, theta, m, v, w, update ? 1 : 0, lr, beta1, beta2, eps, c1, c2);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_pack(const float *theta, const Packed &w, hipStream_t s) {
    hipLaunchKernelGGL(gc_mlp_pack_kernel, dim3((kParams + kThreads - 1) / kThreads), dim3(kThreads), 0, s, theta,
                       w);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_forward(const float *feat, size_t n, const float *theta, const Packed &w, float *logits, uint8_t *cls,
                   hipStream_t s) {
    if (!n) return 0;
    Batch b = {feat, nullptr, nullptr, nullptr, 0, (uint32_t)n, 0.f};
    hipLaunchKernelGGL(gc_mlp_kernel<false>, dim3(groups(n)), dim3(kThreads), kFwdSmem, s, b, theta, w, (float *)nullptr,
                       logits, cls);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace gcmlp
