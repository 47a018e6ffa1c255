// nnp_train.hip -- parameter gradients of a loss L(E, F) for training.
//
// F = -dE/dx (Methods, Eq. 3), so for cotangents gE = dL/dE and gF = dL/dF
//   dL/dW = sum_b gE_b dE_b/dW - d/dW sum_i (dE/dG_i . Gdot_i),
// with Gdot = (dG/dx) gF the AEV tangent (independent of the weights).  Per
// atom and model the inner product is (u/M) times the tangent of the network
// output along Gdot_i, so every network is differentiated through its primal
// and tangent graph with output adjoints alpha = (u/M) gE_b (primal) and
// beta = -u/M (tangent).  This file holds the elementwise layer-3 reverse
// step, the weight-gradient reductions over each element bucket's rows and
// the bias / output-layer sums; the GEMM steps live in nnp_mlp.hip.
#include "nnp_internal.h"

namespace nnp {

template <typename TA> __device__ inline TA dcelu_h_(TA h, TA al) { return h >= TA(0) ? TA(1) : TA(1) + h / al; }

// per-row output adjoints (zero on padding rows)
template <typename TA>
__device__ inline void row_adjoints(int r, const int32_t* __restrict__ atom_of_row,
                                    const int32_t* __restrict__ mol_of_atom,
                                    const double* __restrict__ grad_E, bool has_gF, double scale,
                                    TA& al, TA& be) {
    const int a = atom_of_row[r];
    al = TA(0);
    be = TA(0);
    if (a >= 0) {
        if (grad_E) al = (TA)(scale * grad_E[mol_of_atom[a]]);
        if (has_gF) be = (TA)(-scale);
    }
}

// layer-3 adjoints: zbar3 = w4 (alpha CELU'(z3) + beta (CELU''/CELU')(z3) hdot3),
// zdotbar3 = w4 beta CELU'(z3)
template <typename P>
__global__ __launch_bounds__(256) void k_rev3(int M, int H3, double scale, double celu_alpha,
                                              bool has_gF, const BucketInfo* __restrict__ info,
                                              const int32_t* __restrict__ tile_species, int row_tile,
                                              const int32_t* __restrict__ atom_of_row,
                                              const int32_t* __restrict__ mol_of_atom,
                                              const double* __restrict__ grad_E,
                                              const typename P::TA* __restrict__ w4,
                                              const typename P::TS* __restrict__ Hh,
                                              const typename P::TS* __restrict__ Th,
                                              typename P::TS* __restrict__ ZB,
                                              typename P::TS* __restrict__ ZDB) {
    typedef typename P::TA TA;
    typedef typename P::TS TS;
    const int r = blockIdx.x;
    if (r >= info->rows) return;
    const int s = tile_species[r / row_tile];
    if (s < 0) return;
    TA al, be;
    row_adjoints(r, atom_of_row, mol_of_atom, grad_E, has_gF, scale / M, al, be);
    const TA ca = (TA)celu_alpha;
    const size_t base = (size_t)r * M * H3;
    for (int e = threadIdx.x; e < M * H3; e += blockDim.x) {
        const int m = e / H3, n = e % H3;
        const TA w = w4[((size_t)s * M + m) * H3 + n];
        const TA h = Store<TS>::ld(Hh[base + e]);
        const TA hd = has_gF ? Store<TS>::ld(Th[base + e]) : TA(0);
        const TA d1 = dcelu_h_(h, ca);
        const TA rho = h < TA(0) ? TA(1) / ca : TA(0);
        ZB[base + e] = Store<TS>::st(w * (al * d1 + be * rho * hd));
        ZDB[base + e] = Store<TS>::st(w * be * d1);
    }
}

template <typename P>
hipError_t launch_train_rev3(const Shape& sh, const DevWeights<P>& wt, Work<P>& w,
                             TrainWork<P>& tw, const int32_t* mol_of_atom, const double* grad_E,
                             bool has_gF, hipStream_t st, const Timer& tm) {
    tm.b("train_rev3", st);
    hipLaunchKernelGGL(k_rev3<P>, dim3(sh.Rcap), dim3(256), 0, st, sh.M, sh.H3, sh.energy_scale,
                       sh.celu_alpha, has_gF, w.info, w.tile_species, sh.row_tile, w.atom_of_row,
                       mol_of_atom, grad_E, wt.w4, tw.H3, tw.TH3, w.DZ3, tw.ZDB3);
    tm.e("train_rev3", st);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// Weight gradient of one layer for every (element, model):
//   Wbar[n][k] = sum over the element's bucket rows r of
//                X1[r][xo + n] Y1[r][yo + k] + X2[r][xo + n] Y2[r][yo + k]
// (xo = m * out width, yo = m * in width or 0 for the AEV operands),
// written into the packed gradient array.  MFMA 16x16x4 (FP32 / FP64) takes
// one element per lane, so the row-major tiles feed it without a transpose:
// the reduction runs over rows, 16 per LDS slice.
typedef float f32x4_ __attribute__((ext_vector_type(4)));
typedef double f64x4_ __attribute__((ext_vector_type(4)));
template <typename TS> struct MFW;
template <> struct MFW<float> {
    typedef f32x4_ Acc;
    __device__ static Acc mma(float a, float b, Acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static int row(int l, int r) { return 4 * (l >> 4) + r; }
};
template <> struct MFW<double> {
    typedef f64x4_ Acc;
    __device__ static Acc mma(double a, double b, Acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    __device__ static int row(int l, int r) { return (l >> 4) + 4 * r; }
};

constexpr int kWT = 64;   // output tile (n and k)
constexpr int kWR = 16;   // rows per LDS slice (divides every row tile)

// One workgroup: a 64 x 64 tile of one (element, model) weight gradient,
// 2 x 2 waves of 32 x 32 (many workgroups: the reduction over a bucket's rows
// is serial in each).  The next 16-row slice of both operands is loaded into
// registers (16-byte vectors) while the MFMAs consume the current one from
// LDS.  Columns past an operand's valid width read as zero.
template <typename P>
__global__ __launch_bounds__(256) void k_wgrad(int S, int M, const BucketInfo* __restrict__ info,
                                               const typename P::TS* __restrict__ X1,
                                               const typename P::TS* __restrict__ Y1,
                                               const typename P::TS* __restrict__ X2,
                                               const typename P::TS* __restrict__ Y2, int ldx,
                                               int ldy, int xw, int yw, int out_o, int in_o,
                                               long offW, long net, int ntn,
                                               typename P::TA* __restrict__ gparam) {
    typedef typename P::TS TS;
    typedef typename P::TA TA;
    typedef MFW<TS> mf;
    constexpr int VEC = 16 / (int)sizeof(TS);            // elements per 16-byte load
    constexpr int LD = kWT + VEC;                        // padded LDS row
    constexpr int NV = kWR * kWT / VEC / 256;            // vector loads per thread and operand
    constexpr int FM = kWT / 32, FN = kWT / 32;          // 16 x 16 MFMA tiles per wave
    typedef typename std::conditional<sizeof(TS) == 8, double2, float4>::type TV;
    __shared__ __align__(16) TS Xs[kWR][LD];
    __shared__ __align__(16) TS Ys[kWR][LD];
    const int tile = blockIdx.x, sm = blockIdx.y;
    const int s = sm % S, m = sm / S;
    const int tn = tile % ntn, tk = tile / ntn;
    const int n0 = tn * kWT, k0 = tk * kWT;
    if (n0 >= out_o || k0 >= in_o) return;
    const int r0 = info->off[s], r1 = info->off[s + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int xv = xw, yv = yw ? yw : ldy;               // valid columns of each operand block
    typename mf::Acc acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[i][j][q] = 0;
    const int xo = m * xw + n0, yo = m * yw + k0;
    TV xr[NV], yr[NV];
    auto gload = [&](const TS* X, const TS* Y, int r) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int e = tid + 256 * v, rr = e / (kWT / VEC), col = (e % (kWT / VEC)) * VEC;
            TV zx, zy;
            zx = zy = TV{};
            xr[v] = n0 + col < xv ? *(const TV*)(X + (size_t)(r + rr) * ldx + xo + col) : zx;
            yr[v] = k0 + col < yv ? *(const TV*)(Y + (size_t)(r + rr) * ldy + yo + col) : zy;
        }
    };
    auto lstore = [&]() {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int e = tid + 256 * v, rr = e / (kWT / VEC), col = (e % (kWT / VEC)) * VEC;
            *(TV*)&Xs[rr][col] = xr[v];
            *(TV*)&Ys[rr][col] = yr[v];
        }
    };
    for (int pass = 0; pass < 2; ++pass) {
        const TS* X = pass ? X2 : X1;
        const TS* Y = pass ? Y2 : Y1;
        if (!X || !Y || r0 >= r1) continue;
        gload(X, Y, r0);
        for (int r = r0; r < r1; r += kWR) {
            lstore();
            __syncthreads();
            if (r + kWR < r1) gload(X, Y, r + kWR);
#pragma unroll
            for (int kk = 0; kk < kWR; kk += 4) {
                const int kr = kk + (lane >> 4);
                TS a[FM], b[FN];
#pragma unroll
                for (int i = 0; i < FM; ++i) a[i] = Xs[kr][wm * (kWT / 2) + i * 16 + (lane & 15)];
#pragma unroll
                for (int j = 0; j < FN; ++j) b[j] = Ys[kr][wn * (kWT / 2) + j * 16 + (lane & 15)];
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j) acc[i][j] = mf::mma(a[i], b[j], acc[i][j]);
            }
            __syncthreads();
        }
    }
    TA* out = gparam + ((long)m * S + s) * net + offW;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int n = n0 + wm * (kWT / 2) + i * 16 + mf::row(lane, q);
                const int k = k0 + wn * (kWT / 2) + j * 16 + (lane & 15);
                if (n < out_o && k < in_o) out[(long)n * in_o + k] = (TA)acc[i][j][q];
            }
}

// column sums over each bucket: bias gradients (and, with coefficients, the
// output-layer weights and bias)
template <typename P>
__global__ __launch_bounds__(256) void k_colsum(int S, int M, const BucketInfo* __restrict__ info,
                                                const typename P::TS* __restrict__ X, int ldx, int xw,
                                                int out_o, long offb, long net,
                                                typename P::TA* __restrict__ gparam) {
    typedef typename P::TA TA;
    typedef typename P::TS TS;
    __shared__ TA part[4][64];
    const int sm = blockIdx.y, s = sm % S, m = sm / S;
    const int col = blockIdx.x * 64 + (threadIdx.x & 63), rg = threadIdx.x >> 6;
    TA acc = 0;
    if (col < out_o)
        for (int r = info->off[s] + rg; r < info->off[s + 1]; r += 4)
            acc += Store<TS>::ld(X[(size_t)r * ldx + m * xw + col]);
    part[rg][threadIdx.x & 63] = acc;
    __syncthreads();
    if (rg == 0 && col < out_o)
        gparam[((long)m * S + s) * net + offb + col] =
            (part[0][threadIdx.x] + part[1][threadIdx.x]) + (part[2][threadIdx.x] + part[3][threadIdx.x]);
}

template <typename P>
__global__ __launch_bounds__(256) void k_w4grad(int S, int M, int H3, int o3, double scale,
                                                bool has_gF, const BucketInfo* __restrict__ info,
                                                const int32_t* __restrict__ atom_of_row,
                                                const int32_t* __restrict__ mol_of_atom,
                                                const double* __restrict__ grad_E,
                                                const typename P::TS* __restrict__ Hh,
                                                const typename P::TS* __restrict__ Th, long offw4,
                                                long offb4, long net,
                                                typename P::TA* __restrict__ gparam) {
    typedef typename P::TA TA;
    typedef typename P::TS TS;
    __shared__ TA part[4][64];
    __shared__ TA pb[4][64];
    const int sm = blockIdx.y, s = sm % S, m = sm / S;
    const int col = blockIdx.x * 64 + (threadIdx.x & 63), rg = threadIdx.x >> 6;
    TA acc = 0, accb = 0;
    for (int r = info->off[s] + rg; r < info->off[s + 1]; r += 4) {
        TA al, be;
        row_adjoints(r, atom_of_row, mol_of_atom, grad_E, has_gF, scale / M, al, be);
        if (col < o3) {
            const size_t e = (size_t)r * M * H3 + (size_t)m * H3 + col;
            acc += al * Store<TS>::ld(Hh[e]) + (has_gF ? be * Store<TS>::ld(Th[e]) : TA(0));
        }
        accb += al;
    }
    part[rg][threadIdx.x & 63] = acc;
    pb[rg][threadIdx.x & 63] = accb;
    __syncthreads();
    const int c = threadIdx.x;
    TA* out = gparam + ((long)m * S + s) * net;
    if (rg == 0 && col < o3) out[offw4 + col] = (part[0][c] + part[1][c]) + (part[2][c] + part[3][c]);
    if (threadIdx.x == 0 && blockIdx.x == 0) out[offb4] = (pb[0][0] + pb[1][0]) + (pb[2][0] + pb[3][0]);
}

template <typename P>
hipError_t launch_train_grads(const Shape& sh, const NetLayout& nl, Work<P>& w, TrainWork<P>& tw,
                              const int32_t* mol_of_atom, const double* grad_E, bool has_gF,
                              typename P::TA* gp, hipStream_t st, const Timer& tm) {
    const int S = sh.S, M = sh.M, H1 = sh.H1, H2 = sh.H2, H3 = sh.H3, Dp = sh.Dp;
    const dim3 blk(256);
    tm.b("train_wgrad", st);
    // W3: [o3 x o2] from (ZB3, H2) + (ZDB3, TH2)
    {
        const int ntn = (nl.o3 + kWT - 1) / kWT, ntk = (nl.o2 + kWT - 1) / kWT;
        hipLaunchKernelGGL(k_wgrad<P>, dim3(ntn * ntk, S * M), blk, 0, st, S, M, w.info, w.DZ3,
                           w.H2, has_gF ? tw.ZDB3 : nullptr, tw.TH2, M * H3, M * H2, H3, H2, nl.o3,
                           nl.o2, nl.offW3, nl.net, ntn, gp);
    }
    // W2: [o2 x o1] from (ZB2, H1) + (ZDB2, TH1)
    {
        const int ntn = (nl.o2 + kWT - 1) / kWT, ntk = (nl.o1 + kWT - 1) / kWT;
        hipLaunchKernelGGL(k_wgrad<P>, dim3(ntn * ntk, S * M), blk, 0, st, S, M, w.info, w.DZ2,
                           w.H1, has_gF ? tw.ZDB2 : nullptr, tw.TH1, M * H2, M * H1, H2, H1, nl.o2,
                           nl.o1, nl.offW2, nl.net, ntn, gp);
    }
    // W1: [o1 x D] from (ZB1, G) + (ZDB1, GD)
    {
        const int ntn = (nl.o1 + kWT - 1) / kWT, ntk = (nl.D + kWT - 1) / kWT;
        hipLaunchKernelGGL(k_wgrad<P>, dim3(ntn * ntk, S * M), blk, 0, st, S, M, w.info, w.DZ1,
                           w.G, has_gF ? tw.ZDB1 : nullptr, tw.GD, M * H1, Dp, H1, 0, nl.o1,
                           nl.D, nl.offW1, nl.net, ntn, gp);
    }
    // biases and the output layer
    hipLaunchKernelGGL(k_colsum<P>, dim3((nl.o1 + 63) / 64, S * M), blk, 0, st, S, M, w.info, w.DZ1,
                       M * H1, H1, nl.o1, nl.offb1, nl.net, gp);
    hipLaunchKernelGGL(k_colsum<P>, dim3((nl.o2 + 63) / 64, S * M), blk, 0, st, S, M, w.info, w.DZ2,
                       M * H2, H2, nl.o2, nl.offb2, nl.net, gp);
    hipLaunchKernelGGL(k_colsum<P>, dim3((nl.o3 + 63) / 64, S * M), blk, 0, st, S, M, w.info, w.DZ3,
                       M * H3, H3, nl.o3, nl.offb3, nl.net, gp);
    hipLaunchKernelGGL(k_w4grad<P>, dim3((nl.o3 + 63) / 64, S * M), blk, 0, st, S, M, H3, nl.o3,
                       sh.energy_scale, has_gF, w.info, w.atom_of_row, mol_of_atom, grad_E, tw.H3,
                       tw.TH3, nl.offw4, nl.offb4, nl.net, gp);
    tm.e("train_wgrad", st);
    return hipGetLastError();
}

template <typename TS>
__global__ void k_fill(TS* __restrict__ p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = TS(0);
}

template <typename P>
hipError_t launch_fill(typename P::TS* p, size_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    const size_t blocks = std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill<typename P::TS>, dim3((unsigned)blocks), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

// dL/dx of an energy-only loss: sum_b gE_b dE_b/dx_i = -gE_b(i) F_i
template <typename T>
__global__ void k_grad_coords(int A, const int32_t* __restrict__ mol_of_atom,
                              const double* __restrict__ grad_E, const T* __restrict__ F,
                              T* __restrict__ gx) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 3 * A) return;
    const double g = grad_E ? grad_E[mol_of_atom[i / 3]] : 0.0;
    gx[i] = (T)(-g * (double)F[i]);
}

template <typename P>
hipError_t launch_grad_coords(int A, const int32_t* mol_of_atom, const double* grad_E,
                              const typename P::T* F, typename P::T* gx, hipStream_t st) {
    if (A == 0) return hipSuccess;
    hipLaunchKernelGGL(k_grad_coords<typename P::T>, dim3((3 * A + 255) / 256), dim3(256), 0, st, A,
                       mol_of_atom, grad_E, F, gx);
    return hipGetLastError();
}

// parameter gradients of element networks narrower than the padded layout:
// dst[i] = src[map[i]] (the padded entries are dropped)
template <typename TA>
__global__ void k_gather(int64_t n, const int32_t* __restrict__ map, const TA* __restrict__ src,
                         TA* __restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[map[i]];
}

template <typename TA>
hipError_t launch_gather(int64_t n, const int32_t* map, const TA* src, TA* dst, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather<TA>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, map, src, dst);
    return hipGetLastError();
}
template hipError_t launch_gather<float>(int64_t, const int32_t*, const float*, float*, hipStream_t);
template hipError_t launch_gather<double>(int64_t, const int32_t*, const double*, double*, hipStream_t);

#define NNP_TRAIN_INST(P)                                                                       \
    template hipError_t launch_train_rev3<P>(const Shape&, const DevWeights<P>&, Work<P>&,     \
                                             TrainWork<P>&, const int32_t*, const double*,     \
                                             bool, hipStream_t, const Timer&);                 \
    template hipError_t launch_train_grads<P>(const Shape&, const NetLayout&, Work<P>&,         \
                                              TrainWork<P>&, const int32_t*, const double*,    \
                                              bool, P::TA*, hipStream_t, const Timer&);        \
    template hipError_t launch_fill<P>(P::TS*, size_t, hipStream_t);                           \
    template hipError_t launch_grad_coords<P>(int, const int32_t*, const double*, const P::T*, \
                                              P::T*, hipStream_t);
NNP_TRAIN_INST(PrecF64)
NNP_TRAIN_INST(PrecF32)
template hipError_t launch_fill<PrecBF16>(bf16_t*, size_t, hipStream_t);
template hipError_t launch_grad_coords<PrecBF16>(int, const int32_t*, const double*, const float*,
                                                 float*, hipStream_t);

}  // namespace nnp
