// substrate.hip -- the HyperNEAT substrate layer (the step after the CPPN
// grid queries; the paper supports HyperNEAT, Section 4.3, and the method
// it cites paints a substrate's connection weights with a CPPN).
//
// For every genome g: W[g] is the CPPN's output on all S x S pairs of the
// side x side grid (row p1 = source point, column p2 = target point, the
// order neat_forward_grid writes them in), the expression threshold prunes
// weak weights (|w| < theta -> 0) and the substrate layer maps the shared
// input planes X [B][S] to Y[g] = tanh(X W'[g]) [B][S].
//
// Y[g] = X W'[g] is a dense contraction (M = B, N = K = S), so it runs on
// the matrix cores: v_mfma_f32_16x16x4_f32, fp32 in and fp32 accumulation
// (the precision of the rest of the path).  A workgroup of four waves owns
// a 64 x 64 tile of one genome's Y; K advances in chunks of 32 staged in
// LDS (the threshold is applied as W enters LDS); each wave owns a 32 x 32
// quarter, four 16 x 16 MFMA blocks.  Operand layout of the 16x16x4 MFMA:
// lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16] and receives
// D[4 (l / 16) + r][l % 16] in its r-th accumulator register.
#include <hip/hip_runtime.h>

#include "act.h"
#include "launch.h"

namespace neat {
namespace {

constexpr int ST_M = 64, ST_N = 64, ST_KC = 32;
constexpr int XS_LD = ST_KC + 1;  // padded LDS row strides
constexpr int WS_LD = ST_N + 4;

typedef float f32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void substrate_kernel(SubLaunch L) {
    __shared__ float xs[ST_M * XS_LD];
    __shared__ float ws[ST_KC * WS_LD];
    const int S = L.S, B = L.B;
    const int tiles_m = (B + ST_M - 1) / ST_M, tiles_n = S / ST_N;
    const long long blk = blockIdx.x;
    const int tn = (int)(blk % tiles_n);
    const long long rest = blk / tiles_n;
    const int tm = (int)(rest % tiles_m);
    const long long g = rest / tiles_m;
    const int m0 = tm * ST_M, n0 = tn * ST_N;
    const int t = (int)threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = 32 * (wave >> 1), wn = 32 * (wave & 1);
    const float *Wg = L.W + (size_t)g * S * S;
    const float theta = L.theta;

    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

    // staging assignment: X rows r = t / 4, columns 8 (t % 4) ..; W rows
    // k = t / 8, columns 8 (t % 8) ..
    const int xr = t >> 2, xc = 8 * (t & 3);
    const int wr = t >> 3, wc = 8 * (t & 7);
    const bool xrow_ok = m0 + xr < B;
    for (int k0 = 0; k0 < S; k0 += ST_KC) {
        f32x4 xa = f32x4{0.0f, 0.0f, 0.0f, 0.0f}, xb = xa;
        if (xrow_ok) {
            const f32x4 *src = (const f32x4 *)(L.X + (size_t)(m0 + xr) * S + k0 + xc);
            xa = src[0];
            xb = src[1];
        }
        const f32x4 *wsrc = (const f32x4 *)(Wg + (size_t)(k0 + wr) * S + n0 + wc);
        f32x4 wa = wsrc[0], wb = wsrc[1];
        __syncthreads();  // the previous chunk's reads are done
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            xs[xr * XS_LD + xc + q] = xa[q];
            xs[xr * XS_LD + xc + 4 + q] = xb[q];
            // expression threshold: |w| < theta -> 0 (NaN is kept)
            ws[wr * WS_LD + wc + q] = fabsf(wa[q]) < theta ? 0.0f : wa[q];
            ws[wr * WS_LD + wc + 4 + q] = fabsf(wb[q]) < theta ? 0.0f : wb[q];
        }
        __syncthreads();
        const int li = lane & 15, lk = lane >> 4;
#pragma unroll
        for (int kk = 0; kk < ST_KC; kk += 4) {
            const float a0 = xs[(wm + li) * XS_LD + kk + lk];
            const float a1 = xs[(wm + 16 + li) * XS_LD + kk + lk];
            const float b0 = ws[(kk + lk) * WS_LD + wn + li];
            const float b1 = ws[(kk + lk) * WS_LD + wn + 16 + li];
            acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
        }
    }
    float *Yg = L.Y + (size_t)g * B * S;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
                const int n = n0 + wn + 16 * j + (lane & 15);
                if (m < B) __builtin_nontemporal_store(act_tanh(acc[i][j][r]), Yg + (size_t)m * S + n);
            }
}

}  // namespace

hipError_t substrate_launch(const SubLaunch &L, hipStream_t stream) {
    const long long blocks = (long long)L.P * ((L.B + ST_M - 1) / ST_M) * (L.S / ST_N);
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(substrate_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, L);
    return hipGetLastError();
}

}  // namespace neat
