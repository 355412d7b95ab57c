// Dense layers of the material encoder for one fabric per 256-thread block
// (vectors in LDS, weights row-major in global memory).
#pragma once

#include "common.hpp"

namespace fab {

// y[o] = act(b[o] + sum_i W[o][i] x[i] (+ add[o])) for o < nout.  Each wave
// takes 8 rows at a time so that their weight loads are in flight together;
// per row, lane l sums inputs l, l + 64, ... and a fixed butterfly of wave
// shuffles adds the lanes.  Ends with a block barrier.
__device__ inline void enc_dense_rows(const float *__restrict__ W, const float *__restrict__ b,
                                      const float *x, int nin, int nout, float *y, bool relu,
                                      const float *add)
{
    constexpr int kRows = 8;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nwaves = blockDim.x >> 6;
    for (int o0 = wave * kRows; o0 < nout; o0 += nwaves * kRows) {
        float acc[kRows];
#pragma unroll
        for (int j = 0; j < kRows; j++)
            acc[j] = 0.0f;
        for (int i = lane; i < nin; i += 64) {
            const float xi = x[i];
#pragma unroll
            for (int j = 0; j < kRows; j++)
                if (o0 + j < nout)
                    acc[j] = fmaf(W[(size_t)(o0 + j) * nin + i], xi, acc[j]);
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
                if (o < nout) {
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
// summed over o in order.  Ends with a block barrier.
__device__ inline void enc_dense_cols(const float *__restrict__ W, const float *d, int nout, int nin,
                                      float *y)
{
    for (int i = threadIdx.x; i < nin; i += blockDim.x) {
        float acc = 0.0f;
#pragma unroll 8
        for (int o = 0; o < nout; o++)
            acc = fmaf(W[(size_t)o * nin + i], d[o], acc);
        y[i] = acc;
    }
    __syncthreads();
}

}  // namespace fab
