// gc_mlp.h -- layout and launchers of the selector network kernels
// (40 -> 64 -> 64 -> 16, ReLU, softmax), shared by mlp.hip and the runtime.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace gcmlp {

constexpr int kIn = 40, kInPad = 48, kHid = 64, kOut = 16;
// flat parameter vector: W1[40][64], b1[64], W2[64][64], b2[64], W3[64][16], b3[16]
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kIn * kHid;
constexpr int kOffW2 = kOffB1 + kHid;
constexpr int kOffB2 = kOffW2 + kHid * kHid;
constexpr int kOffW3 = kOffB2 + kHid;
constexpr int kOffB3 = kOffW3 + kHid * kOut;
constexpr int kParams = kOffB3 + kOut;          // 7824
constexpr int kPartialStride = 7840;            // params, loss, padding
constexpr int kRows = 64;                       // samples per workgroup

// bf16 copies of the weights, in the layouts the matrix fragments read
struct Packed {
    uint16_t *w1t;   // [64][48]: W1 transposed, input dim padded with zeros
    uint16_t *w2t;   // [64][64]: W2 transposed
    uint16_t *w2;    // [64][64]: W2
    uint16_t *w3t;   // [16][64]: W3 transposed
    uint16_t *w3;    // [64][16]: W3
};

struct Batch {
    const float *feat;       // rows of 40 features
    const uint32_t *index;   // row of sample r is index[row0 + r] (identity when null)
    const uint8_t *label;    // class of every row
    const float *cost;       // rows of 16 relative size excesses (null when lam == 0)
    size_t row0;
    uint32_t count;          // samples in the batch
    float lam;               // weight of the expected-excess term
};

int launch_grad_partials(const Batch &b, const float *theta, const Packed &w, float *partial, hipStream_t s);
// Sums the partials of `nparts` workgroups; writes the gradient and/or the
// mean loss when asked; with update, one Adam step (c1, c2: the reciprocals
// of the bias corrections) and the bf16 copies.
int launch_reduce_adam(const float *partial, uint32_t nparts, float *grad, float *loss, float *theta, float *m,
                       float *v, const Packed &w, bool update, float lr, float beta1, float beta2, float eps,
                       float c1, float c2, hipStream_t s);
int launch_pack(const float *theta, const Packed &w, hipStream_t s);
int launch_forward(const float *feat, size_t n, const float *theta, const Packed &w, float *logits, uint8_t *cls,
                   hipStream_t s);

}  // namespace gcmlp
