// nnp_params.hip -- device-side replacement of the network parameters.
//
// A training loop keeps its packed master parameters on the GPU (Methods,
// first optimisation: no CPU<->GPU copies per step); this kernel scatters
// them into every device layout the evaluation kernels read (the row-major
// and transposed matrices, the fragment-ordered copies, biases and output
// layer) with the same rounding the host upload applies, so a handle updated
// here computes bitwise what a handle created with the same weights does.
#include "nnp_internal.h"

namespace nnp {

template <typename P, typename TSRC>
__global__ __launch_bounds__(256) void k_set_params(int64_t n, const TSRC* __restrict__ src,
                                                    const int32_t* __restrict__ map, ParamPack pk,
                                                    DevWeights<P> dw) {
    typedef typename P::TS TS;
    typedef typename P::TA TA;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double v = (double)src[i];
    const TS vs = Store<TS>::st((typename P::TA)v);
    const TA va = (TA)v;
    // position in the uniform (padded) packed layout: [m][s]{W1 b1 W2 b2 W3 b3 w4 b4}
    const int64_t pi = map ? (int64_t)map[i] : i;
    const int64_t ms = pi / pk.net;
    const int64_t r = pi - ms * pk.net;
    const int m = (int)(ms / pk.S), s = (int)(ms % pk.S);
    const int M = pk.M, H1 = pk.H1, H2 = pk.H2, H3 = pk.H3, Dp = pk.Dp;
    const size_t sm = (size_t)s * M + m;
    if (r < pk.offb1) {                       // W1 [o1][D]
        const int nn = (int)(r / pk.D), k = (int)(r % pk.D);
        const int col = m * H1 + nn, N1 = M * H1;
        dw.W1[((size_t)s * N1 + col) * Dp + k] = vs;
        dw.W1T[((size_t)s * Dp + k) * N1 + col] = vs;
        if (dw.W1f) {
            dw.W1f[(size_t)s * N1 * Dp + frag_index<TS>(col, k, Dp)] = vs;
            dw.W1Tf[(size_t)s * N1 * Dp + frag_index<TS>(k, col, N1)] = vs;
        }
    } else if (r < pk.offW2) {                // b1 [o1]
        dw.b1[(size_t)s * M * H1 + (size_t)m * H1 + (r - pk.offb1)] = va;
    } else if (r < pk.offb2) {                // W2 [o2][o1]
        const int64_t q = r - pk.offW2;
        const int nn = (int)(q / pk.o1), k = (int)(q % pk.o1);
        dw.W2[(sm * H2 + nn) * H1 + k] = vs;
        dw.W2T[(sm * H1 + k) * H2 + nn] = vs;
        dw.W2f[sm * H2 * H1 + frag_index<TS>(nn, k, H1)] = vs;
        dw.W2Tf[sm * H1 * H2 + frag_index<TS>(k, nn, H2)] = vs;
    } else if (r < pk.offW3) {                // b2 [o2]
        dw.b2[sm * H2 + (r - pk.offb2)] = va;
    } else if (r < pk.offb3) {                // W3 [o3][o2]
        const int64_t q = r - pk.offW3;
        const int nn = (int)(q / pk.o2), k = (int)(q % pk.o2);
        dw.W3[(sm * H3 + nn) * H2 + k] = vs;
        dw.W3T[(sm * H2 + k) * H3 + nn] = vs;
        dw.W3f[sm * H3 * H2 + frag_index<TS>(nn, k, H2)] = vs;
        dw.W3Tf[sm * H2 * H3 + frag_index<TS>(k, nn, H3)] = vs;
    } else if (r < pk.offw4) {                // b3 [o3]
        dw.b3[sm * H3 + (r - pk.offb3)] = va;
    } else if (r < pk.offb4) {                // w4 [o3]
        dw.w4[sm * H3 + (r - pk.offw4)] = va;
    } else {                                  // b4
        dw.b4[sm] = va;
    }
}

template <typename P, typename TSRC>
hipError_t launch_set_params(int64_t n, const TSRC* src, const int32_t* map, const ParamPack& pk,
                             const DevWeights<P>& dw, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_set_params<P, TSRC>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n,
                       src, map, pk, dw);
    return hipGetLastError();
}

#define NNP_SETP(P, TSRC)                                                                          \
    template hipError_t launch_set_params<P, TSRC>(int64_t, const TSRC*, const int32_t*,            \
                                                   const ParamPack&, const DevWeights<P>&, hipStream_t);
NNP_SETP(PrecF64, double)
NNP_SETP(PrecF64, float)
NNP_SETP(PrecF32, double)
NNP_SETP(PrecF32, float)
NNP_SETP(PrecBF16, double)
NNP_SETP(PrecBF16, float)

}  // namespace nnp
