// nnp_mlp.hip -- the ensemble of atomic networks as element-bucketed MFMA GEMMs.
//
// The paper runs all networks of the ensemble and all atoms of a molecule in
// one go instead of one network after another (Methods, third optimisation),
// by replicating each atom's weights in atom order.  Here atoms are instead
// sorted into per-element row buckets across the whole batch, so one element's
// weights serve a tall block of rows, and the M networks of the ensemble are
// fused: layer 1 of all models is one GEMM with the models concatenated along
// N (its backward sums the models along K); layers 2 and 3 run per model
// (grid z).  Per element bucket and row tile:
//
//   L1f  Z1  = G   W1cat^T + b1                 [R x M*H1]
//   L2f  Z2  = celu(Z1_m) W2_m^T + b2            [R x H2]   per model
//   L3f  z3  = celu(Z2_m) W3_m^T + b3;  e_m = w4 . celu(z3) (+ b4 later)
//        DZ3 = celu'(z3) * w4 * gscale            (dE/dz3, gscale = u/M)
//   L3b  DZ2 = (DZ3 W3_m) * celu'(Z2)
//   L2b  DZ1 = (DZ2 W2_m) * celu'(Z1)
//   L1b  dG  = DZ1cat W1cat                      [R x Dp]  (= dE/dAEV)
//
// Operands are K-contiguous in memory (weights as [out][in] for the forward
// and pre-transposed [in][out] copies for the backward), staged through LDS,
// and consumed by 16x16 MFMA tiles: f64 16x16x4, f32 16x16x4, bf16 16x16x32
// (FP32 accumulation).
#include "nnp_internal.h"

namespace nnp {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef short bf16x8 __attribute__((ext_vector_type(8)));

template <typename TS> struct MF;
template <> struct MF<float> {
    static constexpr int KM = 4, KL = 1;
    typedef float Frag;
    typedef f32x4 Acc;
    __device__ static Acc mma(Frag a, Frag b, Acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static Frag ld(const float* p) { return *p; }
    // accumulator element r of lane l holds C[row(l, r)][l % 16]
    __device__ static int row(int l, int r) { return 4 * (l >> 4) + r; }
};
template <> struct MF<double> {
    static constexpr int KM = 4, KL = 1;
    typedef double Frag;
    typedef f64x4 Acc;
    __device__ static Acc mma(Frag a, Frag b, Acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static Frag ld(const double* p) { return *p; }
    // the FP64 16x16x4 accumulator interleaves rows across the lane groups
    __device__ static int row(int l, int r) { return (l >> 4) + 4 * r; }
};
template <> struct MF<bf16_t> {
    static constexpr int KM = 32, KL = 8;
    typedef bf16x8 Frag;
    typedef f32x4 Acc;
    __device__ static Acc mma(Frag a, Frag b, Acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
    __device__ static Frag ld(const bf16_t* p) { return *(const bf16x8*)p; }
    __device__ static int row(int l, int r) { return 4 * (l >> 4) + r; }
};

enum { PRO_NONE = 0, PRO_CELU = 1 };
enum { EPI_BIAS = 0, EPI_L3F = 1, EPI_DSIG = 2, EPI_ACC = 3 };

template <typename TA> __device__ inline TA celu(TA z, TA al) {
    return z >= TA(0) ? z : al * (exp(z / al) - TA(1));
}
__device__ inline float celu(float z, float al) { return z >= 0.f ? z : al * (expf(z / al) - 1.f); }
template <typename TA> __device__ inline TA dcelu(TA z, TA al) { return z >= TA(0) ? TA(1) : exp(z / al); }
__device__ inline float dcelu(float z, float al) { return z >= 0.f ? 1.f : expf(z / al); }

template <typename P> struct GemmArgs {
    typedef typename P::TS TS;
    typedef typename P::TA TA;
    const TS* A; int lda; long a_z;
    const TS* B; int ldb; long b_s, b_z;
    const TA* bias; long bias_s, bias_z;
    void* C; int ldc; long c_z;
    const TS* Zr; int ldz; long z_z;
    const TA* w4; long w4_s, w4_z;
    TA* epart; int n_models, nt;
    TA gscale, alpha;
    int K;
    const int32_t* tile_species; int row_tile;
    const BucketInfo* info;
};

// 16-byte vector of TS elements
template <typename TS> struct Vec16 { static constexpr int N = 16 / sizeof(TS); TS v[N]; };

template <int PRO, typename TS, typename TA>
__device__ inline void prologue(Vec16<TS>& x, TA al) {
    if (PRO == PRO_CELU) {
#pragma unroll
        for (int i = 0; i < Vec16<TS>::N; ++i)
            x.v[i] = Store<TS>::st(celu(Store<TS>::ld(x.v[i]), al));
    }
}

// C tile [BM x BN] of one (row tile, column tile, model).  4 waves laid out
// WM x WN; each wave owns (BM/WM) x (BN/WN) as 16x16 MFMA fragments.
template <typename P, int BM, int BN, int BK, int WM, int WN, int PRO, int EPI>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs<P> g) {
    typedef typename P::TS TS;
    typedef typename P::TA TA;
    typedef MF<TS> mf;
    typedef typename mf::Acc Acc;
    constexpr int WTM = BM / WM, WTN = BN / WN, FM = WTM / 16, FN = WTN / 16;
    static_assert(WM * WN == 4 && FM >= 1 && FN >= 1, "tile");
    constexpr int VE = 16 / sizeof(TS);
    constexpr int PAD = VE;
    constexpr int LDK = BK + PAD;
    __shared__ __align__(16) TS As[BM * LDK];
    __shared__ __align__(16) TS Bs[BN * LDK];

    const int tile_m = blockIdx.x, tile_n = blockIdx.y, z = blockIdx.z;
    const int rows = g.info->rows;
    if (tile_m * BM >= rows) return;
    const int s = g.tile_species[(tile_m * BM) / g.row_tile];
    if (s < 0) return;
    const int tid = threadIdx.x, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave / WN, wn = wave % WN;

    const TS* A = g.A + (size_t)tile_m * BM * g.lda + (size_t)z * g.a_z;
    const TS* B = g.B + (size_t)s * g.b_s + (size_t)z * g.b_z + (size_t)tile_n * BN * g.ldb;

    Acc acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[i][j][r] = 0;

    constexpr int KV = BK / VE;                 // 16B vectors per tile row
    for (int k0 = 0; k0 < g.K; k0 += BK) {
        for (int v = tid; v < BM * KV; v += 256) {
            const int r = v / KV, kc = (v % KV) * VE;
            Vec16<TS> x = *(const Vec16<TS>*)(A + (size_t)r * g.lda + k0 + kc);
            prologue<PRO, TS, TA>(x, g.alpha);
            *(Vec16<TS>*)(As + r * LDK + kc) = x;
        }
        for (int v = tid; v < BN * KV; v += 256) {
            const int r = v / KV, kc = (v % KV) * VE;
            *(Vec16<TS>*)(Bs + r * LDK + kc) = *(const Vec16<TS>*)(B + (size_t)r * g.ldb + k0 + kc);
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < BK; kk += mf::KM) {
            typename mf::Frag af[FM], bfr[FN];
#pragma unroll
            for (int i = 0; i < FM; ++i)
                af[i] = mf::ld(As + (wm * WTM + i * 16 + (lane & 15)) * LDK + kk + (lane >> 4) * mf::KL);
#pragma unroll
            for (int j = 0; j < FN; ++j)
                bfr[j] = mf::ld(Bs + (wn * WTN + j * 16 + (lane & 15)) * LDK + kk + (lane >> 4) * mf::KL);
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j) acc[i][j] = mf::mma(af[i], bfr[j], acc[i][j]);
        }
        __syncthreads();
    }

    // epilogue: fragment element r of lane l is C[mf::row(l, r)][l % 16]
    const int row_base = tile_m * BM + wm * WTM;
    const int col_base = tile_n * BN + wn * WTN + (lane & 15);
    if (EPI == EPI_BIAS) {
        TS* C = (TS*)g.C + (size_t)z * g.c_z;
        const TA* bias = g.bias + (size_t)s * g.bias_s + (size_t)z * g.bias_z;
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int col = col_base + j * 16;
            const TA bb = bias[col];
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = row_base + i * 16 + mf::row(lane, r);
                    C[(size_t)row * g.ldc + col] = Store<TS>::st((TA)acc[i][j][r] + bb);
                }
        }
    } else if (EPI == EPI_ACC) {
        TA* C = (TA*)g.C + (size_t)z * g.c_z;
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    C[(size_t)(row_base + i * 16 + mf::row(lane, r)) * g.ldc + col_base + j * 16] = (TA)acc[i][j][r];
    } else if (EPI == EPI_DSIG) {
        TS* C = (TS*)g.C + (size_t)z * g.c_z;
        const TS* Zr = g.Zr + (size_t)z * g.z_z;
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const size_t row = row_base + i * 16 + mf::row(lane, r);
                    const int col = col_base + j * 16;
                    const TA zz = Store<TS>::ld(Zr[row * g.ldz + col]);
                    C[row * g.ldc + col] = Store<TS>::st((TA)acc[i][j][r] * dcelu(zz, g.alpha));
                }
    } else {   // EPI_L3F
        __shared__ TA red[BM][WN];
        TS* C = (TS*)g.C + (size_t)z * g.c_z;
        const TA* bias = g.bias + (size_t)s * g.bias_s + (size_t)z * g.bias_z;
        const TA* w4 = g.w4 + (size_t)s * g.w4_s + (size_t)z * g.w4_z;
        TA part[FM][4];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) part[i][r] = 0;
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int col = col_base + j * 16;
            const TA bb = bias[col], ww = w4[col];
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = row_base + i * 16 + mf::row(lane, r);
                    const TA zz = (TA)acc[i][j][r] + bb;
                    part[i][r] += ww * celu(zz, g.alpha);
                    C[(size_t)row * g.ldc + col] = Store<TS>::st(dcelu(zz, g.alpha) * ww * g.gscale);
                }
        }
        // sum over the 16 columns held by lanes with equal lane/16
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                TA v = part[i][r];
                v += __shfl_xor(v, 1);
                v += __shfl_xor(v, 2);
                v += __shfl_xor(v, 4);
                v += __shfl_xor(v, 8);
                if ((lane & 15) == 0) red[wm * WTM + i * 16 + mf::row(lane, r)][wn] = v;
            }
        __syncthreads();
        for (int rr = tid; rr < BM; rr += 256) {
            TA v = 0;
#pragma unroll
            for (int q = 0; q < WN; ++q) v += red[rr][q];
            const size_t row = (size_t)tile_m * BM + rr;
            g.epart[(row * g.n_models + z) * g.nt + tile_n] = v;
        }
    }
}

// ---------------------------------------------------------------------------
template <typename P, int BM, int WM, int WN, int PRO, int EPI>
static hipError_t run_gemm(const GemmArgs<P>& a, int Rcap, int N, int nz, hipStream_t st,
                           const Timer& tm, const char* name) {
    constexpr int BN = 64, BK = 32;
    dim3 grid(Rcap / BM, N / BN, nz);
    tm.b(name, st);
    hipLaunchKernelGGL((k_gemm<P, BM, BN, BK, WM, WN, PRO, EPI>), grid, dim3(256), 0, st, a);
    tm.e(name, st);
    return hipGetLastError();
}

template <typename P, int BM, int WM, int WN>
static hipError_t mlp_all(const Shape& sh, const DevWeights<P>& wt, Work<P>& w, hipStream_t st,
                          const Timer& tm) {
    typedef typename P::TA TA;
    const int M = sh.M, H1 = sh.H1, H2 = sh.H2, H3 = sh.H3, Dp = sh.Dp;
    hipError_t e;
    GemmArgs<P> base{};
    base.tile_species = w.tile_species;
    base.row_tile = sh.row_tile;
    base.info = w.info;
    base.alpha = (TA)sh.celu_alpha;
    base.gscale = (TA)(sh.energy_scale / M);
    base.n_models = M;
    base.nt = H3 / 64;

    // L1f
    GemmArgs<P> a = base;
    a.A = w.G; a.lda = Dp; a.a_z = 0;
    a.B = wt.W1; a.ldb = Dp; a.b_s = (long)M * H1 * Dp; a.b_z = 0;
    a.bias = wt.b1; a.bias_s = (long)M * H1; a.bias_z = 0;
    a.C = w.Z1; a.ldc = M * H1; a.c_z = 0;
    a.K = Dp;
    if ((e = run_gemm<P, BM, WM, WN, PRO_NONE, EPI_BIAS>(a, sh.Rcap, M * H1, 1, st, tm, "mlp_l1_fwd")))
        return e;
    // L2f
    a = base;
    a.A = w.Z1; a.lda = M * H1; a.a_z = H1;
    a.B = wt.W2; a.ldb = H1; a.b_s = (long)M * H2 * H1; a.b_z = (long)H2 * H1;
    a.bias = wt.b2; a.bias_s = (long)M * H2; a.bias_z = H2;
    a.C = w.Z2; a.ldc = M * H2; a.c_z = H2;
    a.K = H1;
    if ((e = run_gemm<P, BM, WM, WN, PRO_CELU, EPI_BIAS>(a, sh.Rcap, H2, M, st, tm, "mlp_l2_fwd")))
        return e;
    // L3f (+ output layer, + dE/dz3)
    a = base;
    a.A = w.Z2; a.lda = M * H2; a.a_z = H2;
    a.B = wt.W3; a.ldb = H2; a.b_s = (long)M * H3 * H2; a.b_z = (long)H3 * H2;
    a.bias = wt.b3; a.bias_s = (long)M * H3; a.bias_z = H3;
    a.w4 = wt.w4; a.w4_s = (long)M * H3; a.w4_z = H3;
    a.C = w.DZ3; a.ldc = M * H3; a.c_z = H3;
    a.epart = w.Epart;
    a.K = H2;
    if ((e = run_gemm<P, BM, WM, WN, PRO_CELU, EPI_L3F>(a, sh.Rcap, H3, M, st, tm, "mlp_l3_fwd")))
        return e;
    // L3b
    a = base;
    a.A = w.DZ3; a.lda = M * H3; a.a_z = H3;
    a.B = wt.W3T; a.ldb = H3; a.b_s = (long)M * H2 * H3; a.b_z = (long)H2 * H3;
    a.Zr = w.Z2; a.ldz = M * H2; a.z_z = H2;
    a.C = w.DZ2; a.ldc = M * H2; a.c_z = H2;
    a.K = H3;
    if ((e = run_gemm<P, BM, WM, WN, PRO_NONE, EPI_DSIG>(a, sh.Rcap, H2, M, st, tm, "mlp_l3_bwd")))
        return e;
    // L2b
    a = base;
    a.A = w.DZ2; a.lda = M * H2; a.a_z = H2;
    a.B = wt.W2T; a.ldb = H2; a.b_s = (long)M * H1 * H2; a.b_z = (long)H1 * H2;
    a.Zr = w.Z1; a.ldz = M * H1; a.z_z = H1;
    a.C = w.DZ1; a.ldc = M * H1; a.c_z = H1;
    a.K = H2;
    if ((e = run_gemm<P, BM, WM, WN, PRO_NONE, EPI_DSIG>(a, sh.Rcap, H1, M, st, tm, "mlp_l2_bwd")))
        return e;
    // L1b
    a = base;
    a.A = w.DZ1; a.lda = M * H1; a.a_z = 0;
    a.B = wt.W1T; a.ldb = M * H1; a.b_s = (long)Dp * M * H1; a.b_z = 0;
    a.C = w.dG; a.ldc = Dp; a.c_z = 0;
    a.K = M * H1;
    if ((e = run_gemm<P, BM, WM, WN, PRO_NONE, EPI_ACC>(a, sh.Rcap, Dp, 1, st, tm, "mlp_l1_bwd")))
        return e;
    return hipSuccess;
}

template <typename P>
hipError_t launch_mlp(const Shape& sh, const DevWeights<P>& wt, Work<P>& w, hipStream_t st,
                      const Timer& tm) {
    if (sh.row_tile == 64) return mlp_all<P, 64, 2, 2>(sh, wt, w, st, tm);
    if (sh.row_tile == 16) return mlp_all<P, 16, 1, 4>(sh, wt, w, st, tm);
    return hipErrorInvalidValue;
}

template hipError_t launch_mlp<PrecF64>(const Shape&, const DevWeights<PrecF64>&, Work<PrecF64>&,
                                        hipStream_t, const Timer&);
template hipError_t launch_mlp<PrecF32>(const Shape&, const DevWeights<PrecF32>&, Work<PrecF32>&,
                                        hipStream_t, const Timer&);
template hipError_t launch_mlp<PrecBF16>(const Shape&, const DevWeights<PrecBF16>&,
                                         Work<PrecBF16>&, hipStream_t, const Timer&);

}  // namespace nnp
