// Learned preconditioner: shared definitions of the network kernels.
//
// Network: three 3x3x3 convolutions over an N^3 grid with zero padding,
// 4 -> 16 -> 16 -> 4 channels, relu after the first two. Activations are
// stored channels-last ([cell][channel], cells in z-y-x order, batch
// outermost) in bfloat16; weights as bfloat16 [tap][out][in] with tap
// t = 9 (dz+1) + 3 (dy+1) + (dx+1) reading the cell at offset (dz, dy, dx).
// Products run on the matrix cores (bfloat16 inputs, float32 accumulation).
#pragma once

#include <hip/hip_runtime.h>

namespace rpcg {

constexpr int LP_CIN = 4, LP_HID = 16, LP_COUT = 4, LP_TAPS = 27;
constexpr int LP_W1 = LP_TAPS * LP_HID * LP_CIN;
constexpr int LP_W2 = LP_TAPS * LP_HID * LP_HID;
constexpr int LP_W3 = LP_TAPS * LP_COUT * LP_HID;
// flat parameter vector: W1 b1 W2 b2 W3 b3
constexpr int LP_OFF_W1 = 0, LP_OFF_B1 = LP_W1, LP_OFF_W2 = LP_OFF_B1 + LP_HID, LP_OFF_B2 = LP_OFF_W2 + LP_W2,
              LP_OFF_W3 = LP_OFF_B2 + LP_HID, LP_OFF_B3 = LP_OFF_W3 + LP_W3, LP_NPARAMS = LP_OFF_B3 + LP_COUT;

typedef unsigned short bf16_t;
typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// float32 -> bfloat16, nearest with ties to even (finite inputs).
__host__ __device__ __forceinline__ bf16_t f32_to_bf16(float f)
{
    const unsigned b = __builtin_bit_cast(unsigned, f);
    return (bf16_t)((b + 0x7FFFu + ((b >> 16) & 1u)) >> 16);
}

__host__ __device__ __forceinline__ float bf16_to_f32(bf16_t h)
{
    return __builtin_bit_cast(float, (unsigned)h << 16);
}

enum { EPI_RELU = 0, EPI_LINEAR = 1, EPI_MASK = 2 };

// ---- launchers (lp_conv.hip) ----
// out = conv(in) with prepared weights wt [27][16][CIN] (bfloat16, output
// channels padded to 16). EPI_RELU: act (bfloat16 [cell][COUT]) =
// relu(acc + bias), and pre (float32, when not null) = acc + bias.
// EPI_LINEAR: pre = acc + bias. EPI_MASK: act = acc where the forward
// activation mask (bfloat16 [cell][COUT], the relu layer's output) is
// nonzero, else 0 (the adjoint pass of a relu layer).
hipError_t launch_lp_conv(int cin, int cout, int epi, int nb, int N, const bf16_t *in, const bf16_t *wt,
                          const float *bias, const bf16_t *mask, float *pre, bf16_t *act, hipStream_t s);
// Partial weight and bias gradients in grid slots (one workgroup of three
// wavefronts per slot): pw[g][27][16][16] (out, in), pb[g][16]; then a
// fixed-order sum over the slots.
hipError_t launch_lp_conv_dw(int cin, int cout, int nb, int N, const bf16_t *in, const bf16_t *dout, float *pw,
                             float *pb, int grid, hipStream_t s);
hipError_t launch_lp_reduce(int nslots, int cout, int cin, const float *pw, const float *pb, float *gw, float *gb,
                            hipStream_t s);
// Weight preparation from the float32 parameters: forward copies and the
// transposed, tap-mirrored copies of layers 2 and 3 for the adjoint passes.
hipError_t launch_lp_prep(const float *params, bf16_t *w1, bf16_t *w2, bf16_t *w3, bf16_t *w2t, bf16_t *w3t,
                          hipStream_t s);
hipError_t launch_lp_adam(int n, float *params, const float *grad, float *m, float *v, float lr, float b1, float b2,
                          float eps, int step, hipStream_t s);

} // namespace rpcg
