// Dense layers of the material encoder for one fabric per block
// (vectors in LDS, weights row-major in global memory).
#pragma once

#include "common.hpp"

namespace fab {

// sum over k < n of a[k * as] * b[k * bs] (b null: of a[k * as] * 1), added
// in the order k = 0, 1, ..., with the loads of eight consecutive terms
// issued together (n is a run-time count, so a plain loop would wait for
// memory once per term).
__device__ inline float ordered_dot(const float *__restrict__ a, int as,
                                    const float *__restrict__ b, int bs, int n)
{
    float acc = 0.0f;
    for (int k0 = 0; k0 < n; k0 += 8) {
        float av[8], bv[8];
#pragma unroll
        for (int j = 0; j < 8; j++) {
            const size_t k = k0 + j < n ? k0 + j : k0;
            av[j] = a[k * as];
            bv[j] = b ? b[k * bs] : 1.0f;
        }
#pragma unroll
        for (int j = 0; j < 8; j++)
            if (k0 + j < n)
                acc = fmaf(av[j], bv[j], acc);
    }
    return acc;
}

// Threads of an encoder block: 16 waves, so that one round of 8 rows per
// wave covers a hidden layer's 128 outputs.
constexpr int kEncThreads = 1024;

// y[o] = act(b[o] + sum_i W[o][i] x[i] (+ add[o])) for o < NOUT.  Each wave
// takes 8 rows at a time; per row, lane l sums inputs l, l + 64, ... in
// order and a fixed butterfly of wave shuffles adds the lanes.  The fan-in
// is a compile-time constant, so that all of a lane's weight loads for its 8
// rows are issued before the first product (the layer waits for memory
// once, not once per 64 inputs).  Ends with a block barrier.
template <int NIN, int NOUT>
__device__ inline void enc_dense_rows(const float *__restrict__ W, const float *__restrict__ b,
                                      const float *x, float *y, bool relu, const float *add)
{
    constexpr int kRows = 8;
    constexpr int kPer = (NIN + 63) / 64;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nwaves = blockDim.x >> 6;
    for (int o0 = wave * kRows; o0 < NOUT; o0 += nwaves * kRows) {
        float w[kRows][kPer];
#pragma unroll
        for (int j = 0; j < kRows; j++)
#pragma unroll
            for (int k = 0; k < kPer; k++) {
                const int i = lane + 64 * k;
                w[j][k] = o0 + j < NOUT && i < NIN ? W[(size_t)(o0 + j) * NIN + i] : 0.0f;
            }
        float acc[kRows];
#pragma unroll
        for (int j = 0; j < kRows; j++)
            acc[j] = 0.0f;
#pragma unroll
        for (int k = 0; k < kPer; k++) {
            const int i = lane + 64 * k;
            if (i < NIN) {
                const float xi = x[i];
#pragma unroll
                for (int j = 0; j < kRows; j++)
                    acc[j] = fmaf(w[j][k], xi, acc[j]);
            }
        }
#pragma unroll
        for (int j = 0; j < kRows; j++) {
#pragma unroll
            for (int off = 32; off > 0; off >>= 1)
                acc[j] += __shfl_xor(acc[j], off, 64);
        }
        if (lane == 0) {
#pragma unroll
            for (int j = 0; j < kRows; j++) {
                const int o = o0 + j;
                if (o < NOUT) {
                    float val = acc[j] + b[o];
                    if (add)
                        val += add[o];
                    y[o] = relu ? fmaxf(val, 0.0f) : val;
                }
            }
        }
    }
    __syncthreads();
}

// y[i] = sum_o W[o][i] d[o] (the transposed product), one output per thread,
// summed over o in order; the loads of 32 consecutive o are issued together.
// Ends with a block barrier.
template <int NOUT, int NIN>
__device__ inline void enc_dense_cols(const float *__restrict__ W, const float *d, float *y)
{
    constexpr int kBatch = NOUT < 32 ? NOUT : 32;
    static_assert(NOUT % kBatch == 0, "whole batches");
    for (int i = threadIdx.x; i < NIN; i += blockDim.x) {
        float acc = 0.0f;
#pragma unroll 1
        for (int o0 = 0; o0 < NOUT; o0 += kBatch) {
            float w[kBatch];
#pragma unroll
            for (int o = 0; o < kBatch; o++)
                w[o] = W[(size_t)(o0 + o) * NIN + i];
#pragma unroll
            for (int o = 0; o < kBatch; o++)
                acc = fmaf(w[o], d[o0 + o], acc);
        }
        y[i] = acc;
    }
    __syncthreads();
}

// The encoder for a latent of LAT values (32: the config-size network, 64:
// the paper-size network's encoder): layers E1 .. E3 as above, then E4
// [LAT][128] and c4 [LAT].
template <int LAT> constexpr int enc_off_c4() { return kOffE4 + LAT * kEncHid; }
template <int LAT> constexpr int enc_param_count() { return enc_off_c4<LAT>() + LAT; }
// Per-fabric backward scratch: x[524] e1 r2 e2 d1 d2 d3 [128 each] dz[LAT].
template <int LAT> constexpr int enc_act_floats() { return kEncIn + 6 * kEncHid + LAT; }

// Forward of one fabric by one block of kEncThreads:
// e1 = relu(E1 x + c1), e2 = relu(e1 + E3 relu(E2 e1 + c2) + c3), z = E4 e2 + c4.
template <int LAT>
__device__ inline void encoder_forward_block(const float *__restrict__ Q, const float *__restrict__ in,
                                             float *__restrict__ z_out)
{
    __shared__ float x[kEncIn];
    __shared__ float e1[kEncHid], r2[kEncHid], e2[kEncHid], z[LAT];
    for (int k = threadIdx.x; k < kEncIn; k += blockDim.x)
        x[k] = in[k];
    __syncthreads();
    enc_dense_rows<kEncIn, kEncHid>(Q + kOffE1, Q + kOffC1, x, e1, true, nullptr);
    enc_dense_rows<kEncHid, kEncHid>(Q + kOffE2, Q + kOffC2, e1, r2, true, nullptr);
    enc_dense_rows<kEncHid, kEncHid>(Q + kOffE3, Q + kOffC3, r2, e2, true, e1);
    enc_dense_rows<kEncHid, LAT>(Q + kOffE4, Q + enc_off_c4<LAT>(), e2, z, false, nullptr);
    for (int k = threadIdx.x; k < LAT; k += blockDim.x)
        z_out[k] = z[k];
}

// Backward of one fabric by one block of kEncThreads: recompute the forward,
// backpropagate dz to the layers' pre-activation gradients and store the
// inputs and gradients the weight gradients need (layout of enc_act_floats).
template <int LAT>
__device__ inline void encoder_backward_block(const float *__restrict__ Q, const float *__restrict__ in,
                                              const float *__restrict__ dz, float *__restrict__ out)
{
    __shared__ float x[kEncIn], a1[kEncHid], e1[kEncHid], a2[kEncHid], r2[kEncHid],
        a3[kEncHid], e2[kEncHid], g[kEncHid], d3[kEncHid], d2[kEncHid], d1[kEncHid], dzs[LAT];
    for (int k = threadIdx.x; k < kEncIn; k += blockDim.x)
        x[k] = in[k];
    for (int k = threadIdx.x; k < LAT; k += blockDim.x)
        dzs[k] = dz[k];
    __syncthreads();
    enc_dense_rows<kEncIn, kEncHid>(Q + kOffE1, Q + kOffC1, x, a1, false, nullptr);
    for (int k = threadIdx.x; k < kEncHid; k += blockDim.x)
        e1[k] = fmaxf(a1[k], 0.0f);
    __syncthreads();
    enc_dense_rows<kEncHid, kEncHid>(Q + kOffE2, Q + kOffC2, e1, a2, false, nullptr);
    for (int k = threadIdx.x; k < kEncHid; k += blockDim.x)
        r2[k] = fmaxf(a2[k], 0.0f);
    __syncthreads();
    enc_dense_rows<kEncHid, kEncHid>(Q + kOffE3, Q + kOffC3, r2, a3, false, nullptr);
    for (int k = threadIdx.x; k < kEncHid; k += blockDim.x) {
        a3[k] += e1[k];                     // skip connection before the activation
        e2[k] = fmaxf(a3[k], 0.0f);
    }
    __syncthreads();
    enc_dense_cols<LAT, kEncHid>(Q + kOffE4, dzs, g);              // dL/de2
    for (int k = threadIdx.x; k < kEncHid; k += blockDim.x)
        d3[k] = a3[k] > 0.0f ? g[k] : 0.0f;
    __syncthreads();
    enc_dense_cols<kEncHid, kEncHid>(Q + kOffE3, d3, g);           // dL/dr2
    for (int k = threadIdx.x; k < kEncHid; k += blockDim.x)
        d2[k] = a2[k] > 0.0f ? g[k] : 0.0f;
    __syncthreads();
    enc_dense_cols<kEncHid, kEncHid>(Q + kOffE2, d2, g);           // dL/de1 (through E2)
    for (int k = threadIdx.x; k < kEncHid; k += blockDim.x)
        d1[k] = a1[k] > 0.0f ? g[k] + d3[k] : 0.0f;               // plus the skip path
    __syncthreads();
    for (int k = threadIdx.x; k < kEncIn; k += blockDim.x)
        out[k] = x[k];
    for (int k = threadIdx.x; k < kEncHid; k += blockDim.x) {
        out[kEncIn + k] = e1[k];
        out[kEncIn + kEncHid + k] = r2[k];
        out[kEncIn + 2 * kEncHid + k] = e2[k];
        out[kEncIn + 3 * kEncHid + k] = d1[k];
        out[kEncIn + 4 * kEncHid + k] = d2[k];
        out[kEncIn + 5 * kEncHid + k] = d3[k];
    }
    for (int k = threadIdx.x; k < LAT; k += blockDim.x)
        out[kEncIn + 6 * kEncHid + k] = dzs[k];
}

// Encoder parameter e's gradient: the sum over fabrics, in order, of the
// products of its layer's output gradient and input in the scratch of
// encoder_backward_block.
template <int LAT>
__device__ inline float encoder_wgrad_entry(const float *__restrict__ scratch, int n_fabrics, int e)
{
    constexpr int kAct = enc_act_floats<LAT>();
    constexpr int kC4 = enc_off_c4<LAT>();
    // (delta offset, input offset, fan-in) of the tensor holding e
    int dofs, xofs, nin, idx;
    if (e < kOffC1) { dofs = kEncIn + 3 * kEncHid; xofs = 0; nin = kEncIn; idx = e - kOffE1; }
    else if (e < kOffE2) { dofs = kEncIn + 3 * kEncHid; xofs = -1; nin = 1; idx = e - kOffC1; }
    else if (e < kOffC2) { dofs = kEncIn + 4 * kEncHid; xofs = kEncIn; nin = kEncHid; idx = e - kOffE2; }
    else if (e < kOffE3) { dofs = kEncIn + 4 * kEncHid; xofs = -1; nin = 1; idx = e - kOffC2; }
    else if (e < kOffC3) { dofs = kEncIn + 5 * kEncHid; xofs = kEncIn + kEncHid; nin = kEncHid; idx = e - kOffE3; }
    else if (e < kOffE4) { dofs = kEncIn + 5 * kEncHid; xofs = -1; nin = 1; idx = e - kOffC3; }
    else if (e < kC4) { dofs = kEncIn + 6 * kEncHid; xofs = kEncIn + 2 * kEncHid; nin = kEncHid; idx = e - kOffE4; }
    else { dofs = kEncIn + 6 * kEncHid; xofs = -1; nin = 1; idx = e - kC4; }
    const int o = idx / nin, i = idx % nin;
    return ordered_dot(scratch + dofs + o, kAct, xofs >= 0 ? scratch + xofs + i : nullptr, kAct,
                       n_fabrics);
}

}  // namespace fab
