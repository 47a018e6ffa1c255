// nnp_mlp.hip -- the ensemble of atomic networks as element-bucketed MFMA GEMMs.
//
// The paper runs all networks of the ensemble and all atoms of a molecule in
// one go instead of one network after another (Methods, third optimisation),
// by replicating each atom's weights in atom order.  Here atoms are instead
// sorted into per-element row buckets across the whole batch, so one element's
// weights serve a tall block of rows, and the M networks of the ensemble are
// fused: layer 1 of all models is one GEMM with the models concatenated along
// N (its backward sums the models along K); layers 2 and 3 run per model.
// Per element bucket and row tile (h = CELU(z), CELU'(z) = 1 + min(h, 0)/alpha):
//
//   L1f  H1  = celu(G W1cat^T + b1)               [R x M*H1]
//   L2f  H2  = celu(H1_m W2_m^T + b2)             [R x H2]   per model
//   L3f  z3  = H2_m W3_m^T + b3;  e_m = w4 . celu(z3) (+ b4 later)
//        DZ3 = celu'(z3) * w4 * gscale            (dE/dz3, gscale = u/M)
//   L3b  DZ2 = (DZ3 W3_m) * celu'(H2)
//   L2b  DZ1 = (DZ2 W2_m) * celu'(H1)
//   L1b  dG  = DZ1cat W1cat                       [R x Dp]  (= dE/dAEV)
//
// Operands are K-contiguous in memory (weights as [out][in] for the forward
// and pre-transposed [in][out] copies for the backward).  Each workgroup of 4
// waves owns a BM x BN output tile; K is streamed in BK slices through a
// double-buffered LDS tile (the next slice is fetched into registers while the
// current one feeds the MFMAs); bf16 slices are 128-byte rows whose 16-byte
// chunks are XOR-swizzled by row so fragment reads and tile writes hit
// distinct banks.  MFMA: f64 16x16x4, f32 16x16x4, bf16 16x16x32 (FP32
// accumulation).  Tiles are scheduled N-fastest and remapped so each XCD
// works through a contiguous range (its L2 keeps the row block and the
// weights it shares).
#include <algorithm>

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
    __device__ static int row(int l, int r) { return 4 * (l >> 4) + r; }
};

// LDS layout of a [rows][BK] operand slice.  off(r, c) = element offset of
// the 16-byte chunk c of row r; frag(r, k) = offset of the fragment that
// starts at column k.
template <typename TS, int BK> struct Tile {
    static constexpr int VE = 16 / sizeof(TS);          // elements per 16-byte chunk
    static constexpr int CH = BK / VE;                  // chunks per row
    static constexpr int LD = BK + VE;                  // padded row (non-bf16)
    static constexpr int size(int rows) { return rows * LD; }
    __device__ static int off(int r, int c) { return r * LD + c * VE; }
    __device__ static int frag(int r, int k) { return r * LD + k; }
};
template <int BK> struct Tile<bf16_t, BK> {
    static constexpr int VE = 8;
    static constexpr int CH = BK / VE;
    static_assert((CH & (CH - 1)) == 0, "chunks per row must be a power of two");
    static constexpr int size(int rows) { return rows * BK; }
    __device__ static int off(int r, int c) { return r * BK + ((c ^ (r & (CH - 1))) << 3); }
    __device__ static int frag(int r, int k) { return off(r, k >> 3); }
};

enum { EPI_CELU = 0, EPI_L3F = 1, EPI_DSIG = 2, EPI_ACC = 3, EPI_RAW = 4, EPI_REV = 5 };

__device__ inline float celu(float z, float al) {
    return z >= 0.f ? z : al * (__builtin_amdgcn_exp2f(z * (1.44269504088896341f / al)) - 1.f);
}
__device__ inline double celu(double z, double al) { return z >= 0.0 ? z : al * expm1(z / al); }
__device__ inline float dcelu_z(float z, float al) {
    return z >= 0.f ? 1.f : __builtin_amdgcn_exp2f(z * (1.44269504088896341f / al));
}
__device__ inline double dcelu_z(double z, double al) { return z >= 0.0 ? 1.0 : exp(z / al); }
// CELU'(z) from h = CELU(z): h >= 0 <=> z >= 0, and exp(z/alpha) = 1 + h/alpha
template <typename TA> __device__ inline TA dcelu_h(TA h, TA al) { return h >= TA(0) ? TA(1) : TA(1) + h / al; }

template <typename P> struct GemmArgs {
    typedef typename P::TS TS;
    typedef typename P::TA TA;
    const TS* A; int lda; long a_z;
    const TS* B; int ldb; long b_s, b_z;
    const TA* bias; long bias_s, bias_z;
    void* C; int ldc; long c_z;
    const TS* Hr; int ldh; long h_z;        // stored activations for CELU'
    void* C2; long c2_z;                     // second output (EPI_REV), leading dim ldc
    const TS* X; int ldx; long x_z;          // auxiliary product (EPI_REV)
    const TS* Tr; int ldt; long t_z;         // tangent activations (EPI_REV)
    const TA* w4; long w4_s, w4_z;
    TA* epart; int n_models, nt;
    TA gscale, alpha;
    int K;
    const int32_t* tile_species; int row_tile;
    const BucketInfo* info;
    int nm, nn, nz;                          // tiles along M, N and models
};

typedef int i32x4 __attribute__((ext_vector_type(4)));   // one 16-byte chunk

// Row tiles are grouped kGroupM at a time: within a group the schedule runs
// M-fastest, so the tiles an XCD has in flight share both a few row blocks
// and a few weight column blocks in its L2.
constexpr int kGroupM = 8;

template <typename P, int BM, int BN, int BK, int WM, int WN>
struct GemmShape {
    typedef typename P::TS TS;
    typedef Tile<TS, BK> L;
    static constexpr size_t lds_bytes() {
        return sizeof(TS) * 2 * ((size_t)L::size(BM) + (size_t)L::size(BN)) +
               sizeof(typename P::TA) * BM * WN;
    }
};

template <typename P, int BM, int BN, int BK, int WM, int WN, int EPI>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs<P> g) {
    typedef typename P::TS TS;
    typedef typename P::TA TA;
    typedef MF<TS> mf;
    typedef typename mf::Acc Acc;
    typedef Tile<TS, BK> L;
    constexpr int WTM = BM / WM, WTN = BN / WN, FM = WTM / 16, FN = WTN / 16;
    static_assert(WM * WN == 4 && FM >= 1 && FN >= 1, "tile");
    constexpr int NVA = BM * L::CH, NVB = BN * L::CH;          // 16-byte chunks per slice
    constexpr int RA = (NVA + 255) / 256, RB = (NVB + 255) / 256;
    extern __shared__ __align__(16) char smem_raw[];
    TS* As0 = (TS*)smem_raw;
    TS* As1 = As0 + L::size(BM);
    TS* Bs0 = As1 + L::size(BM);
    TS* Bs1 = Bs0 + L::size(BN);
    TA* red = (TA*)(Bs1 + L::size(BN));                         // [BM][WN] (L3F only)

    // ---- tile schedule.  Block ids are dealt round-robin to the 8 XCDs;
    // XCD x gets the contiguous logical range it would own in order, and
    // that range is walked group by group (kGroupM row tiles, M-fastest).
    const int T = g.nm * g.nn * g.nz;
    const int bid = blockIdx.x, xcd = bid & 7, slot = bid >> 3;
    const int q8 = T >> 3, r8 = T & 7;
    const int lin = xcd * q8 + (xcd < r8 ? xcd : r8) + slot;
    const int per_z = g.nm * g.nn;
    const int z = lin / per_z, rem = lin % per_z;
    const int grp = rem / (kGroupM * g.nn), inside = rem % (kGroupM * g.nn);
    const int gsz = min(kGroupM, g.nm - grp * kGroupM);
    const int tile_n = inside / gsz, tile_m = grp * kGroupM + inside % gsz;

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

    // two register sets of prefetched K slices (slice k+2 is fetched while
    // slice k is consumed and slice k+1 is parked in LDS)
    i32x4 pa0[RA], pb0[RB], pa1[RA], pb1[RB];
#define NNP_FETCH(PA, PB, kslice)                                                             \
    {                                                                                         \
        const int k0_ = (kslice) * BK;                                                        \
        _Pragma("unroll") for (int u = 0; u < RA; ++u) {                                      \
            const int v = tid + 256 * u;                                                      \
            if (v < NVA)                                                                      \
                PA[u] = *(const i32x4*)(A + (size_t)(v / L::CH) * g.lda + k0_ + (v % L::CH) * L::VE); \
        }                                                                                     \
        _Pragma("unroll") for (int u = 0; u < RB; ++u) {                                      \
            const int v = tid + 256 * u;                                                      \
            if (v < NVB)                                                                      \
                PB[u] = *(const i32x4*)(B + (size_t)(v / L::CH) * g.ldb + k0_ + (v % L::CH) * L::VE); \
        }                                                                                     \
    }
#define NNP_STASH(PA, PB, AS, BS)                                                             \
    {                                                                                         \
        _Pragma("unroll") for (int u = 0; u < RA; ++u) {                                      \
            const int v = tid + 256 * u;                                                      \
            if (v < NVA) *(i32x4*)(&AS[L::off(v / L::CH, v % L::CH)]) = PA[u];                \
        }                                                                                     \
        _Pragma("unroll") for (int u = 0; u < RB; ++u) {                                      \
            const int v = tid + 256 * u;                                                      \
            if (v < NVB) *(i32x4*)(&BS[L::off(v / L::CH, v % L::CH)]) = PB[u];                \
        }                                                                                     \
    }
#define NNP_COMPUTE(AS, BS)                                                                   \
    {                                                                                         \
        _Pragma("unroll") for (int kk = 0; kk < BK; kk += mf::KM) {                          \
            typename mf::Frag af[FM];                                                         \
            const int kf = kk + (lane >> 4) * mf::KL;                                         \
            _Pragma("unroll") for (int i = 0; i < FM; ++i)                                    \
                af[i] = *(const typename mf::Frag*)(&AS[L::frag(wm * WTM + i * 16 + (lane & 15), kf)]); \
            _Pragma("unroll") for (int j = 0; j < FN; ++j) {                                  \
                const typename mf::Frag bfr =                                                 \
                    *(const typename mf::Frag*)(&BS[L::frag(wn * WTN + j * 16 + (lane & 15), kf)]); \
                _Pragma("unroll") for (int i = 0; i < FM; ++i)                                \
                    acc[i][j] = mf::mma(af[i], bfr, acc[i][j]);                               \
            }                                                                                 \
        }                                                                                     \
    }

    const int nk = g.K / BK;
    NNP_FETCH(pa0, pb0, 0)
    if (nk > 1) NNP_FETCH(pa1, pb1, 1)
    NNP_STASH(pa0, pb0, As0, Bs0)
    __syncthreads();
    for (int kt = 0; kt < nk; kt += 2) {
        // even slice kt in buffer 0; slice kt+1 waits in (pa1, pb1)
        if (kt + 2 < nk) NNP_FETCH(pa0, pb0, kt + 2)
        NNP_COMPUTE(As0, Bs0)
        if (kt + 1 < nk) NNP_STASH(pa1, pb1, As1, Bs1)
        __syncthreads();
        if (kt + 1 >= nk) break;
        // odd slice kt+1 in buffer 1; slice kt+2 waits in (pa0, pb0)
        if (kt + 3 < nk) NNP_FETCH(pa1, pb1, kt + 3)
        NNP_COMPUTE(As1, Bs1)
        if (kt + 2 < nk) NNP_STASH(pa0, pb0, As0, Bs0)
        __syncthreads();
    }
#undef NNP_FETCH
#undef NNP_STASH
#undef NNP_COMPUTE

    // ---- epilogue: fragment element r of lane l is C[mf::row(l, r)][l % 16]
    const int row_base = tile_m * BM + wm * WTM;
    const int col_base = tile_n * BN + wn * WTN + (lane & 15);
    if (EPI == EPI_CELU) {
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
                    C[(size_t)row * g.ldc + col] = Store<TS>::st(celu((TA)acc[i][j][r] + bb, g.alpha));
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
                    C[(size_t)(row_base + i * 16 + mf::row(lane, r)) * g.ldc + col_base + j * 16] =
                        (TA)acc[i][j][r];
    } else if (EPI == EPI_DSIG) {
        TS* C = (TS*)g.C + (size_t)z * g.c_z;
        const TS* Hr = g.Hr + (size_t)z * g.h_z;
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const size_t row = row_base + i * 16 + mf::row(lane, r);
                    const int col = col_base + j * 16;
                    const TA hh = Store<TS>::ld(Hr[row * g.ldh + col]);
                    C[row * g.ldc + col] = Store<TS>::st((TA)acc[i][j][r] * dcelu_h(hh, g.alpha));
                }
    } else if (EPI == EPI_RAW) {
        TS* C = (TS*)g.C + (size_t)z * g.c_z;
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    C[(size_t)(row_base + i * 16 + mf::row(lane, r)) * g.ldc + col_base + j * 16] =
                        Store<TS>::st((TA)acc[i][j][r]);
    } else if (EPI == EPI_REV) {
        // reverse step through h = CELU(z) and its tangent hdot = CELU'(z) zdot:
        //   zbar    = abar CELU'(z) + acheck (CELU''/CELU')(z) hdot
        //   zdotbar = acheck CELU'(z)
        // abar = this product, acheck = X (the same product of the tangent
        // adjoint), CELU''/CELU' = 1/alpha for z < 0 and 0 otherwise.
        TS* C = (TS*)g.C + (size_t)z * g.c_z;
        TS* C2 = (TS*)g.C2 + (size_t)z * g.c2_z;
        const TS* Hr = g.Hr + (size_t)z * g.h_z;
        const TS* X = g.X + (size_t)z * g.x_z;
        const TS* Tr = g.Tr + (size_t)z * g.t_z;
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const size_t row = row_base + i * 16 + mf::row(lane, r);
                    const int col = col_base + j * 16;
                    const TA hh = Store<TS>::ld(Hr[row * g.ldh + col]);
                    const TA ac = Store<TS>::ld(X[row * g.ldx + col]);
                    const TA hd = Store<TS>::ld(Tr[row * g.ldt + col]);
                    const TA d1 = dcelu_h(hh, g.alpha);
                    const TA rho = hh < TA(0) ? TA(1) / g.alpha : TA(0);
                    C[row * g.ldc + col] = Store<TS>::st((TA)acc[i][j][r] * d1 + ac * rho * hd);
                    C2[row * g.ldc + col] = Store<TS>::st(ac * d1);
                }
    } else {   // EPI_L3F
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
                    C[(size_t)row * g.ldc + col] = Store<TS>::st(dcelu_z(zz, g.alpha) * ww * g.gscale);
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
                if ((lane & 15) == 0) red[(wm * WTM + i * 16 + mf::row(lane, r)) * WN + wn] = v;
            }
        __syncthreads();
        for (int rr = tid; rr < BM; rr += 256) {
            TA v = 0;
#pragma unroll
            for (int q = 0; q < WN; ++q) v += red[rr * WN + q];
            const size_t row = (size_t)tile_m * BM + rr;
            g.epart[(row * g.n_models + z) * g.nt + tile_n] = v;
        }
    }
}

// ---------------------------------------------------------------------------
template <typename P, int BM, int BN, int BK, int WM, int WN, int EPI>
static hipError_t run_gemm(GemmArgs<P> a, int Rcap, int N, int nz, hipStream_t st,
                           const Timer& tm, const char* name) {
    a.nm = Rcap / BM;
    a.nn = N / BN;
    a.nz = nz;
    const int T = a.nm * a.nn * a.nz;
    const size_t lds = GemmShape<P, BM, BN, BK, WM, WN>::lds_bytes();
    auto kern = k_gemm<P, BM, BN, BK, WM, WN, EPI>;
    hipError_t e = ensure_lds((const void*)kern, lds);
    if (e != hipSuccess) return e;
    tm.b(name, st);
    hipLaunchKernelGGL(kern, dim3(T), dim3(256), lds, st, a);
    tm.e(name, st);
    return hipGetLastError();
}

// tile shapes per precision and row tile: BM = row tile; wide N tiles for
// the layer-1 GEMMs, 64-wide for the per-model layers (widths 192 / 256)
template <typename P, int BM> struct Cfg;
template <> struct Cfg<PrecBF16, 128> {
    static constexpr int BK = 64, BNW = 128, BNN = 64, WM = 2, WN = 2;
};
template <> struct Cfg<PrecF32, 128> {
    static constexpr int BK = 32, BNW = 128, BNN = 64, WM = 2, WN = 2;
};
template <> struct Cfg<PrecF64, 128> {
    static constexpr int BK = 16, BNW = 64, BNN = 64, WM = 2, WN = 2;
};
template <typename P> struct Cfg<P, 16> {
    static constexpr int BK = sizeof(typename P::TS) == 2 ? 64 : (sizeof(typename P::TS) == 4 ? 32 : 16);
    static constexpr int BNW = 64, BNN = 64, WM = 1, WN = 4;
};

template <typename P, int BM>
static hipError_t mlp_all(const Shape& sh, const DevWeights<P>& wt, Work<P>& w, hipStream_t st,
                          const Timer& tm) {
    typedef typename P::TA TA;
    typedef Cfg<P, BM> C;
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
    const int R = sh.Rcap;

    // L1f
    GemmArgs<P> a = base;
    a.A = w.G; a.lda = Dp; a.a_z = 0;
    a.B = wt.W1; a.ldb = Dp; a.b_s = (long)M * H1 * Dp; a.b_z = 0;
    a.bias = wt.b1; a.bias_s = (long)M * H1; a.bias_z = 0;
    a.C = w.H1; a.ldc = M * H1; a.c_z = 0;
    a.K = Dp;
    if ((M * H1) % C::BNW == 0)
        e = run_gemm<P, BM, C::BNW, C::BK, C::WM, C::WN, EPI_CELU>(a, R, M * H1, 1, st, tm, "mlp_l1_fwd");
    else
        e = run_gemm<P, BM, C::BNN, C::BK, C::WM, C::WN, EPI_CELU>(a, R, M * H1, 1, st, tm, "mlp_l1_fwd");
    if (e) return e;
    // L2f
    a = base;
    a.A = w.H1; a.lda = M * H1; a.a_z = H1;
    a.B = wt.W2; a.ldb = H1; a.b_s = (long)M * H2 * H1; a.b_z = (long)H2 * H1;
    a.bias = wt.b2; a.bias_s = (long)M * H2; a.bias_z = H2;
    a.C = w.H2; a.ldc = M * H2; a.c_z = H2;
    a.K = H1;
    if ((e = run_gemm<P, BM, C::BNN, C::BK, C::WM, C::WN, EPI_CELU>(a, R, H2, M, st, tm, "mlp_l2_fwd")))
        return e;
    // L3f (+ output layer, + dE/dz3)
    a = base;
    a.A = w.H2; a.lda = M * H2; a.a_z = H2;
    a.B = wt.W3; a.ldb = H2; a.b_s = (long)M * H3 * H2; a.b_z = (long)H3 * H2;
    a.bias = wt.b3; a.bias_s = (long)M * H3; a.bias_z = H3;
    a.w4 = wt.w4; a.w4_s = (long)M * H3; a.w4_z = H3;
    a.C = w.DZ3; a.ldc = M * H3; a.c_z = H3;
    a.epart = w.Epart;
    a.K = H2;
    if ((e = run_gemm<P, BM, 64, C::BK, C::WM, C::WN, EPI_L3F>(a, R, H3, M, st, tm, "mlp_l3_fwd")))
        return e;
    // L3b
    a = base;
    a.A = w.DZ3; a.lda = M * H3; a.a_z = H3;
    a.B = wt.W3T; a.ldb = H3; a.b_s = (long)M * H2 * H3; a.b_z = (long)H2 * H3;
    a.Hr = w.H2; a.ldh = M * H2; a.h_z = H2;
    a.C = w.DZ2; a.ldc = M * H2; a.c_z = H2;
    a.K = H3;
    if ((e = run_gemm<P, BM, C::BNN, C::BK, C::WM, C::WN, EPI_DSIG>(a, R, H2, M, st, tm, "mlp_l3_bwd")))
        return e;
    // L2b
    a = base;
    a.A = w.DZ2; a.lda = M * H2; a.a_z = H2;
    a.B = wt.W2T; a.ldb = H2; a.b_s = (long)M * H1 * H2; a.b_z = (long)H1 * H2;
    a.Hr = w.H1; a.ldh = M * H1; a.h_z = H1;
    a.C = w.DZ1; a.ldc = M * H1; a.c_z = H1;
    a.K = H2;
    if (H1 % C::BNW == 0)
        e = run_gemm<P, BM, C::BNW, C::BK, C::WM, C::WN, EPI_DSIG>(a, R, H1, M, st, tm, "mlp_l2_bwd");
    else
        e = run_gemm<P, BM, C::BNN, C::BK, C::WM, C::WN, EPI_DSIG>(a, R, H1, M, st, tm, "mlp_l2_bwd");
    if (e) return e;
    // L1b
    a = base;
    a.A = w.DZ1; a.lda = M * H1; a.a_z = 0;
    a.B = wt.W1T; a.ldb = M * H1; a.b_s = (long)Dp * M * H1; a.b_z = 0;
    a.C = w.dG; a.ldc = Dp; a.c_z = 0;
    a.K = M * H1;
    if (Dp % C::BNW == 0)
        e = run_gemm<P, BM, C::BNW, C::BK, C::WM, C::WN, EPI_ACC>(a, R, Dp, 1, st, tm, "mlp_l1_bwd");
    else
        e = run_gemm<P, BM, C::BNN, C::BK, C::WM, C::WN, EPI_ACC>(a, R, Dp, 1, st, tm, "mlp_l1_bwd");
    return e;
}

// ---------------------------------------------------------------------------
// Training: forward with the layer-3 activations kept, the tangent forward
// along the AEV tangent GD, and the reverse pass through the primal and
// tangent graph down to the layer-1 adjoints (weight gradients are formed in
// nnp_train.hip from the buffers left here).
template <typename P, int BM>
static hipError_t train_mlp(const Shape& sh, const DevWeights<P>& wt, Work<P>& w, TrainWork<P>& tw,
                            const int32_t* mol_of_atom, const double* grad_E, bool has_gF,
                            hipStream_t st, const Timer& tm) {
    typedef typename P::TA TA;
    typedef Cfg<P, BM> C;
    constexpr int BN = C::BNN;
    const int M = sh.M, H1 = sh.H1, H2 = sh.H2, H3 = sh.H3, Dp = sh.Dp;
    const int R = sh.Rcap;
    hipError_t e;
    GemmArgs<P> base{};
    base.tile_species = w.tile_species;
    base.row_tile = sh.row_tile;
    base.info = w.info;
    base.alpha = (TA)sh.celu_alpha;
    base.gscale = (TA)(sh.energy_scale / M);
    base.n_models = M;
    base.nt = H3 / 64;
    GemmArgs<P> a;
#define NNP_RUN(EPI, N, NZ, NAME)                                                               \
    if ((e = run_gemm<P, BM, BN, C::BK, C::WM, C::WN, EPI>(a, R, N, NZ, st, tm, NAME))) return e;

    // forward: H1, H2, H3
    a = base;
    a.A = w.G; a.lda = Dp; a.B = wt.W1; a.ldb = Dp; a.b_s = (long)M * H1 * Dp;
    a.bias = wt.b1; a.bias_s = (long)M * H1; a.C = w.H1; a.ldc = M * H1; a.K = Dp;
    NNP_RUN(EPI_CELU, M * H1, 1, "train_l1_fwd")
    a = base;
    a.A = w.H1; a.lda = M * H1; a.a_z = H1;
    a.B = wt.W2; a.ldb = H1; a.b_s = (long)M * H2 * H1; a.b_z = (long)H2 * H1;
    a.bias = wt.b2; a.bias_s = (long)M * H2; a.bias_z = H2;
    a.C = w.H2; a.ldc = M * H2; a.c_z = H2; a.K = H1;
    NNP_RUN(EPI_CELU, H2, M, "train_l2_fwd")
    a = base;
    a.A = w.H2; a.lda = M * H2; a.a_z = H2;
    a.B = wt.W3; a.ldb = H2; a.b_s = (long)M * H3 * H2; a.b_z = (long)H3 * H2;
    a.bias = wt.b3; a.bias_s = (long)M * H3; a.bias_z = H3;
    a.C = tw.H3; a.ldc = M * H3; a.c_z = H3; a.K = H2;
    NNP_RUN(EPI_CELU, H3, M, "train_l3_fwd")
    // tangent forward: TH_l = CELU'(z_l) (TH_{l-1} W_l^T)
    if (has_gF) {
        a = base;
        a.A = tw.GD; a.lda = Dp; a.B = wt.W1; a.ldb = Dp; a.b_s = (long)M * H1 * Dp;
        a.Hr = w.H1; a.ldh = M * H1; a.C = tw.TH1; a.ldc = M * H1; a.K = Dp;
        NNP_RUN(EPI_DSIG, M * H1, 1, "train_l1_tan")
        a = base;
        a.A = tw.TH1; a.lda = M * H1; a.a_z = H1;
        a.B = wt.W2; a.ldb = H1; a.b_s = (long)M * H2 * H1; a.b_z = (long)H2 * H1;
        a.Hr = w.H2; a.ldh = M * H2; a.h_z = H2; a.C = tw.TH2; a.ldc = M * H2; a.c_z = H2; a.K = H1;
        NNP_RUN(EPI_DSIG, H2, M, "train_l2_tan")
        a = base;
        a.A = tw.TH2; a.lda = M * H2; a.a_z = H2;
        a.B = wt.W3; a.ldb = H2; a.b_s = (long)M * H3 * H2; a.b_z = (long)H3 * H2;
        a.Hr = tw.H3; a.ldh = M * H3; a.h_z = H3; a.C = tw.TH3; a.ldc = M * H3; a.c_z = H3; a.K = H2;
        NNP_RUN(EPI_DSIG, H3, M, "train_l3_tan")
    }
    return hipSuccess;
}

// reverse propagation below layer 3 (layer-3 adjoints are elementwise and
// written by nnp_train.hip into DZ3 / ZDB3 first)
template <typename P, int BM>
static hipError_t train_mlp_rev(const Shape& sh, const DevWeights<P>& wt, Work<P>& w,
                                TrainWork<P>& tw, hipStream_t st, const Timer& tm) {
    typedef typename P::TA TA;
    typedef Cfg<P, BM> C;
    constexpr int BN = C::BNN;
    const int M = sh.M, H1 = sh.H1, H2 = sh.H2, H3 = sh.H3;
    const int R = sh.Rcap;
    hipError_t e;
    GemmArgs<P> base{};
    base.tile_species = w.tile_species;
    base.row_tile = sh.row_tile;
    base.info = w.info;
    base.alpha = (TA)sh.celu_alpha;
    base.n_models = M;
    GemmArgs<P> a;
    const int ldt = M * (H1 > H2 ? H1 : H2);
    // layer 2 adjoints: acheck2 = ZDB3 W3, abar2 = ZB3 W3
    a = base;
    a.A = tw.ZDB3; a.lda = M * H3; a.a_z = H3;
    a.B = wt.W3T; a.ldb = H3; a.b_s = (long)M * H2 * H3; a.b_z = (long)H2 * H3;
    a.C = tw.TMP; a.ldc = ldt; a.c_z = H2; a.K = H3;
    NNP_RUN(EPI_RAW, H2, M, "train_l3_rev_t")
    a = base;
    a.A = w.DZ3; a.lda = M * H3; a.a_z = H3;
    a.B = wt.W3T; a.ldb = H3; a.b_s = (long)M * H2 * H3; a.b_z = (long)H2 * H3;
    a.Hr = w.H2; a.ldh = M * H2; a.h_z = H2;
    a.X = tw.TMP; a.ldx = ldt; a.x_z = H2;
    a.Tr = tw.TH2; a.ldt = M * H2; a.t_z = H2;
    a.C = w.DZ2; a.C2 = tw.ZDB2; a.ldc = M * H2; a.c_z = H2; a.c2_z = H2; a.K = H3;
    NNP_RUN(EPI_REV, H2, M, "train_l3_rev")
    // layer 1 adjoints
    a = base;
    a.A = tw.ZDB2; a.lda = M * H2; a.a_z = H2;
    a.B = wt.W2T; a.ldb = H2; a.b_s = (long)M * H1 * H2; a.b_z = (long)H1 * H2;
    a.C = tw.TMP; a.ldc = ldt; a.c_z = H1; a.K = H2;
    NNP_RUN(EPI_RAW, H1, M, "train_l2_rev_t")
    a = base;
    a.A = w.DZ2; a.lda = M * H2; a.a_z = H2;
    a.B = wt.W2T; a.ldb = H2; a.b_s = (long)M * H1 * H2; a.b_z = (long)H1 * H2;
    a.Hr = w.H1; a.ldh = M * H1; a.h_z = H1;
    a.X = tw.TMP; a.ldx = ldt; a.x_z = H1;
    a.Tr = tw.TH1; a.ldt = M * H1; a.t_z = H1;
    a.C = w.DZ1; a.C2 = tw.ZDB1; a.ldc = M * H1; a.c_z = H1; a.c2_z = H1; a.K = H2;
    NNP_RUN(EPI_REV, H1, M, "train_l2_rev")
#undef NNP_RUN
    return hipSuccess;
}

template <typename P>
hipError_t launch_train_mlp(const Shape& sh, const DevWeights<P>& wt, Work<P>& w,
                            TrainWork<P>& tw, const int32_t* mol_of_atom, const double* grad_E,
                            bool has_gF, hipStream_t st, const Timer& tm) {
    if (sh.row_tile == 128) return train_mlp<P, 128>(sh, wt, w, tw, mol_of_atom, grad_E, has_gF, st, tm);
    if (sh.row_tile == 16) return train_mlp<P, 16>(sh, wt, w, tw, mol_of_atom, grad_E, has_gF, st, tm);
    return hipErrorInvalidValue;
}

template <typename P>
hipError_t launch_train_mlp_rev(const Shape& sh, const DevWeights<P>& wt, Work<P>& w,
                                TrainWork<P>& tw, hipStream_t st, const Timer& tm) {
    if (sh.row_tile == 128) return train_mlp_rev<P, 128>(sh, wt, w, tw, st, tm);
    if (sh.row_tile == 16) return train_mlp_rev<P, 16>(sh, wt, w, tw, st, tm);
    return hipErrorInvalidValue;
}

template <typename P>
hipError_t launch_mlp(const Shape& sh, const DevWeights<P>& wt, Work<P>& w, hipStream_t st,
                      const Timer& tm) {
    if (sh.row_tile == 128) return mlp_all<P, 128>(sh, wt, w, st, tm);
    if (sh.row_tile == 16) return mlp_all<P, 16>(sh, wt, w, st, tm);
    return hipErrorInvalidValue;
}

#define NNP_TRAIN_INST(P)                                                                   \
    template hipError_t launch_train_mlp<P>(const Shape&, const DevWeights<P>&, Work<P>&,       \
                                            TrainWork<P>&, const int32_t*, const double*, bool, \
                                            hipStream_t, const Timer&);                          \
    template hipError_t launch_train_mlp_rev<P>(const Shape&, const DevWeights<P>&, Work<P>&,   \
                                                TrainWork<P>&, hipStream_t, const Timer&);
NNP_TRAIN_INST(PrecF64)
NNP_TRAIN_INST(PrecF32)

template hipError_t launch_mlp<PrecF64>(const Shape&, const DevWeights<PrecF64>&, Work<PrecF64>&,
                                        hipStream_t, const Timer&);
template hipError_t launch_mlp<PrecF32>(const Shape&, const DevWeights<PrecF32>&, Work<PrecF32>&,
                                        hipStream_t, const Timer&);
template hipError_t launch_mlp<PrecBF16>(const Shape&, const DevWeights<PrecBF16>&,
                                         Work<PrecBF16>&, hipStream_t, const Timer&);

}  // namespace nnp
