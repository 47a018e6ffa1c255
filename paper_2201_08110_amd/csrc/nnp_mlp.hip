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
#include <type_traits>

#include "nnp_internal.h"

namespace nnp {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef short bf16x8 __attribute__((ext_vector_type(8)));

template <typename TS> struct MF;
template <> struct MF<float> {
    static constexpr int KM = 4, KL = 1;   // K of one MFMA, K elements per lane
    typedef float Frag;
    typedef f32x4 Acc;
    __device__ static Acc mma(Frag a, Frag b, Acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // with the operands swapped (B fragment first) accumulator element r of
    // lane l holds C[l % 16][col0(l) + r * kColStride]
    static constexpr int kColStride = 1;
    __device__ static int col0(int l) { return 4 * (l >> 4); }
};
template <> struct MF<double> {
    static constexpr int KM = 4, KL = 1;
    typedef double Frag;
    typedef f64x4 Acc;
    __device__ static Acc mma(Frag a, Frag b, Acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // the FP64 16x16x4 accumulator interleaves its rows across the lane
    // groups, so a lane's four elements are every fourth column
    static constexpr int kColStride = 4;
    __device__ static int col0(int l) { return l >> 4; }
};
template <> struct MF<bf16_t> {
    static constexpr int KM = 32, KL = 8;
    typedef bf16x8 Frag;
    typedef f32x4 Acc;
    __device__ static Acc mma(Frag a, Frag b, Acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
    static constexpr int kColStride = 1;
    __device__ static int col0(int l) { return 4 * (l >> 4); }
};

// LDS layout of one K slice of an operand: [rows][128 bytes], i.e. BK =
// 128 / sizeof(TS) elements per row in eight 16-byte chunks; chunk c of row r
// sits at position c ^ (r & 7), so the sixteen rows a fragment read touches
// and the eight rows one direct-to-LDS load writes spread over all banks.
template <typename TS> struct Slice {
    static constexpr int VE = 16 / (int)sizeof(TS);     // elements per chunk
    static constexpr int BK = 8 * VE;                   // elements per row
    __device__ static int at(int r, int k) { return r * BK + ((((k / VE) ^ r) & 7) * VE) + (k % VE); }
};

// Fragments of G consecutive k-steps read as one 16-byte vector per lane
// (element j feeds step j): four FP32 or two FP64 k-steps; a BF16 fragment
// already fills 16 bytes.
template <typename TS> struct FragGroup {
    static constexpr int G = 1;
    typedef typename MF<TS>::Frag V;
    __device__ static typename MF<TS>::Frag at(const V& v, int) { return v; }
};
template <> struct FragGroup<float> {
    static constexpr int G = 4;
    typedef f32x4 V;
    __device__ static float at(const V& v, int j) { return v[j]; }
};
typedef double f64x2 __attribute__((ext_vector_type(2)));
template <> struct FragGroup<double> {
    static constexpr int G = 2;
    typedef f64x2 V;
    __device__ static double at(const V& v, int j) { return v[j]; }
};

enum { EPI_CELU = 0, EPI_L3F = 1, EPI_DSIG = 2, EPI_ACC = 3, EPI_RAW = 4, EPI_REV = 5 };

// CELU and its derivative, branch-free (the exponential is taken of min(z, 0)
// and always finite); ial = 1 / alpha.  CELU'(z) is recovered from a stored
// h = CELU(z): h >= 0 <=> z >= 0, and exp(z / alpha) = 1 + h / alpha.
// (float: the scaled argument is clamped, min(z c, 0) = min(z, 0) c for c > 0,
// so the minimum takes a product and needs no NaN canonicalisation of z)
__device__ inline float celu(float z, float al, float ial) {
    const float e = __builtin_amdgcn_exp2f(fminf(z * (ial * 1.44269504088896341f), 0.f));
    return z >= 0.f ? z : __builtin_fmaf(al, e, -al);
}
__device__ inline double celu(double z, double al, double ial) {
    const double e = expm1(fmin(z, 0.0) * ial);
    return z >= 0.0 ? z : al * e;
}
__device__ inline float dcelu_z(float z, float ial) {
    // exp2 of the clamped argument is exactly 1 for z >= 0
    return __builtin_amdgcn_exp2f(fminf(z * (ial * 1.44269504088896341f), 0.f));
}
__device__ inline double dcelu_z(double z, double ial) {
    const double e = exp(fmin(z, 0.0) * ial);
    return z >= 0.0 ? 1.0 : e;
}
// (1 + h / alpha >= 1 exactly when h >= 0, so the minimum selects the branch)
__device__ inline float dcelu_h(float h, float ial) { return fminf(__builtin_fmaf(h, ial, 1.f), 1.f); }
__device__ inline double dcelu_h(double h, double ial) { return h >= 0.0 ? 1.0 : 1.0 + h * ial; }

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
    TA gscale, alpha, inv_alpha;
    int K;
    const int32_t* tile_species; int row_tile;
    const BucketInfo* info;
    int nm, nn, nz;                          // tiles along M, N and models
};

// Four output elements of one row held by one lane: columns c, c+ST, c+2ST,
// c+3ST (ST = 1 for the f32 / bf16 MFMAs, 4 for f64).
template <typename TS, int ST> struct Quad {
    typedef typename std::conditional<sizeof(TS) == 8, double, float>::type TA;
    __device__ static void ld(const TS* p, TA v[4]) {
#pragma unroll
        for (int r = 0; r < 4; ++r) v[r] = Store<TS>::ld(p[r * ST]);
    }
    __device__ static void st(TS* p, const TA v[4]) {
#pragma unroll
        for (int r = 0; r < 4; ++r) p[r * ST] = Store<TS>::st(v[r]);
    }
};
template <> struct Quad<float, 1> {
    __device__ static void ld(const float* p, float v[4]) {
        const float4 q = *(const float4*)p;
        v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
    }
    __device__ static void st(float* p, const float v[4]) { *(float4*)p = make_float4(v[0], v[1], v[2], v[3]); }
};
template <> struct Quad<bf16_t, 1> {
    __device__ static void ld(const bf16_t* p, float v[4]) {
        const uint2 q = *(const uint2*)p;
        v[0] = bf2f((bf16_t)(q.x & 0xffffu)); v[1] = bf2f((bf16_t)(q.x >> 16));
        v[2] = bf2f((bf16_t)(q.y & 0xffffu)); v[3] = bf2f((bf16_t)(q.y >> 16));
    }
    __device__ static void st(bf16_t* p, const float v[4]) {
        uint2 q;
        q.x = pack_bf16x2(v[0], v[1]);
        q.y = pack_bf16x2(v[2], v[3]);
        *(uint2*)p = q;
    }
};

// Store one 16-row x 64-column BF16 strip held in the MFMA accumulator
// layout (lane l: row l%16; piece j = columns 16 j + 4 (l/16) .. +3, packed
// as two BF16 pairs pk[j][0..1]) so that each store instruction writes 64
// contiguous bytes per row instead of 32: the four lanes of a row trade
// pieces (ds_bpermute) until lane q holds columns 8q..8q+7 and 32+8q..32+8q+7.
// p points at (row l%16, column 8 (l/16)) of the strip.  Fewer, wider write
// requests make these stores markedly cheaper on gfx950.
__device__ inline void st_strip_bf16(bf16_t* p, const uint32_t (&pk)[4][2], int lane) {
    const int q = lane >> 4, hi = q >> 1, odd = q & 1;
    // sources: lanes (l%16) + 32 (q%2) and 16 past it.  Odd q pulls them in
    // the other order, so the 32 lanes of each ds_bpermute read 32 distinct
    // banks (lane (l%16) + 32 and lane l%16 would share one).
    const int srcA = ((lane & 15) + 32 * odd) * 4, srcB = srcA + 64;   // byte lane addresses
    const int s1 = odd ? srcB : srcA, s2 = odd ? srcA : srcB;
#pragma unroll
    for (int h = 0; h < 2; ++h) {   // columns 32 h + 8 q ..: piece 2 h + q/2 of lanes 2(q%2), 2(q%2)+1
        const int jl = 2 * h, jh = 2 * h + 1;
        uint32_t a0 = __builtin_amdgcn_ds_bpermute(s1, (int)pk[jl][0]);
        uint32_t a1 = __builtin_amdgcn_ds_bpermute(s1, (int)pk[jh][0]);
        uint32_t b0 = __builtin_amdgcn_ds_bpermute(s1, (int)pk[jl][1]);
        uint32_t b1 = __builtin_amdgcn_ds_bpermute(s1, (int)pk[jh][1]);
        const uint32_t f0 = hi ? a1 : a0, f1 = hi ? b1 : b0;   // from s1
        a0 = __builtin_amdgcn_ds_bpermute(s2, (int)pk[jl][0]);
        a1 = __builtin_amdgcn_ds_bpermute(s2, (int)pk[jh][0]);
        b0 = __builtin_amdgcn_ds_bpermute(s2, (int)pk[jl][1]);
        b1 = __builtin_amdgcn_ds_bpermute(s2, (int)pk[jh][1]);
        const uint32_t g0 = hi ? a1 : a0, g1 = hi ? b1 : b0;   // from s2
        uint4 o;
        o.x = odd ? g0 : f0;   // columns +0..3 come from srcA
        o.y = odd ? g1 : f1;
        o.z = odd ? f0 : g0;   // columns +4..7 from srcB
        o.w = odd ? f1 : g1;
        *(uint4*)(p + 32 * h) = o;
    }
}

// Row tiles are grouped kGroupM at a time: within a group the schedule runs
// M-fastest, so the tiles an XCD has in flight share both a few row blocks
// and a few weight column blocks in its L2.
constexpr int kGroupM = 8;

template <typename P, int BM, int BN, int WM, int WN, int S>
struct GemmShape {
    typedef typename P::TS TS;
    static constexpr size_t lds_bytes() {
        return (size_t)S * (BM + BN) * 128 + sizeof(typename P::TA) * BM * WN;
    }
};

#define NNP_GPTR(p) ((const void __attribute__((address_space(1)))*)(p))
#define NNP_LPTR(p) ((void __attribute__((address_space(3)))*)(p))

// Wait until at most N of this wave's vector-memory operations are still in
// flight and all its LDS operations have completed, then meet the other
// waves.  Direct-to-LDS loads count as vector-memory operations and complete
// in issue order, so N = loads issued for later slices leaves exactly those
// in flight.  The memory clobber keeps the compiler from moving LDS accesses
// across the barrier (a plain __syncthreads would wait for every load).
template <int N> __device__ inline void vm_wait_barrier() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    // s_waitcnt vmcnt(N) expcnt(7) lgkmcnt(0), issued through the builtin so
    // that the compiler's own wait tracking sees it
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4));
    asm volatile("s_barrier" ::: "memory");
}
// s_waitcnt vmcnt(N) alone (expcnt and lgkmcnt left at their maxima)
template <int N> __device__ inline void vm_wait() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// One workgroup of 4 waves computes a BM x BN tile of C = A B^T (A [rows][K],
// B [N][K], both K-contiguous).  K streams through S LDS stages of 128-byte
// rows, filled by direct global->LDS loads (no register staging) issued S-1
// slices ahead.  The MFMA operands are swapped (B fragment first), so every
// lane ends up owning four columns of one output row and the epilogue reads
// and writes 8- or 16-byte vectors.
template <typename P, int BM, int BN, int WM, int WN, int S, int EPI>
__global__ __launch_bounds__(64 * WM * WN) void k_gemm(GemmArgs<P> g) {
    typedef typename P::TS TS;
    typedef typename P::TA TA;
    typedef MF<TS> mf;
    typedef typename mf::Acc Acc;
    typedef Slice<TS> L;
    constexpr int BK = L::BK;
    constexpr int WTM = BM / WM, WTN = BN / WN, FM = WTM / 16, FN = WTN / 16;
    constexpr int NW = WM * WN;                            // waves per workgroup
    static_assert((NW == 4 || NW == 8) && FM >= 1 && FN >= 1, "tile");
    static_assert(S >= 2 && BM % 8 == 0 && BN % 8 == 0, "stages / rows");
    constexpr int NQA = BM / 8, NQB = BN / 8;              // 8-row (1 KiB) loads per slice
    constexpr int QA = (NQA + NW - 1) / NW, QB = (NQB + NW - 1) / NW;   // per wave (at most)
    constexpr int QMIN = NQA / NW + NQB / NW;                            // per wave (at least)
    constexpr int ST = mf::kColStride;
    extern __shared__ __align__(16) char smem_raw[];
    TS* const stage0 = (TS*)smem_raw;                      // stage s: A rows then B rows
    TA* red = (TA*)(smem_raw + (size_t)S * (BM + BN) * 128);   // [BM][WN] (L3F only)

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
    const int tid = threadIdx.x, lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wm = wave / WN, wn = wave % WN;

    const TS* A = g.A + (size_t)tile_m * BM * g.lda + (size_t)z * g.a_z;
    const TS* B = g.B + (size_t)s * g.b_s + (size_t)z * g.b_z + (size_t)tile_n * BN * g.ldb;

    // this lane's part of every 8-row load: row lane/8 of the group, the
    // chunk that lands at position lane%8 of it
    const int ld_row = lane >> 3, ld_chunk = (lane & 7) ^ (lane >> 3);
    // direct loads of K slice `src` into LDS stage `slot`
    auto issue = [&](int src, int slot) {
        TS* st_ = stage0 + (size_t)slot * (BM + BN) * BK;
        const int k0 = src * BK + ld_chunk * L::VE;
#pragma unroll
        for (int u = 0; u < QA; ++u) {
            const int q = wave + NW * u;
            if (NQA % NW == 0 || q < NQA)
                __builtin_amdgcn_global_load_lds(NNP_GPTR(A + (size_t)(q * 8 + ld_row) * g.lda + k0),
                                                 NNP_LPTR(st_ + q * 8 * BK), 16, 0, 0);
        }
#pragma unroll
        for (int u = 0; u < QB; ++u) {
            const int q = wave + NW * u;
            if (NQB % NW == 0 || q < NQB)
                __builtin_amdgcn_global_load_lds(NNP_GPTR(B + (size_t)(q * 8 + ld_row) * g.ldb + k0),
                                                 NNP_LPTR(st_ + (BM + q * 8) * BK), 16, 0, 0);
        }
    };

    Acc acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[i][j][r] = 0;

    // Software pipeline: the fragments of k-step t+1 are read from LDS while
    // the MFMAs of step t run; the last step of a slice first waits for the
    // next slice and the barrier that frees the oldest stage, refills that
    // stage, then reads the next slice's first fragments.  Every step issues
    // the same number of direct loads (past the end the last slice is loaded
    // again into the free stage, an L2 hit), so one wait count fits all steps
    // and the loop body has no branches (a join would make the compiler wait
    // for every LDS read).  Scheduling barriers keep the compiler from
    // moving the MFMAs of a step above the reads issued for the next one.
    // FP32 / FP64 fragments hold one element per lane and k-step, so a
    // plain read would fetch 4 or 8 bytes per lane.  Those are read FG
    // k-steps at a time instead, one 16-byte chunk per lane: within a group,
    // lane group g holds k = kk + g FG + j for step j, which still covers
    // kk .. kk + 4 FG - 1 once each, identically for A and B (only the order
    // of the K sum changes).
    typedef typename FragGroup<TS>::V FragG;
    constexpr int FG = FragGroup<TS>::G, KG = mf::KM * FG;   // k-steps, K per group
    constexpr int NSTEP = BK / KG;
    static_assert(NSTEP % 2 == 0, "k-step groups per slice");
    auto stage = [&](int kt) { return stage0 + (size_t)(kt % S) * (BM + BN) * BK; };
    FragG af[2][FM], bq[2][FN];
    auto read_frags = [&](FragG(&fa)[FM], FragG(&fb)[FN], const TS* As, int kk) {
        const TS* Bs = As + BM * BK;
        const int kf = kk + (lane >> 4) * mf::KL * FG;
#pragma unroll
        for (int i = 0; i < FM; ++i) fa[i] = *(const FragG*)(&As[L::at(wm * WTM + i * 16 + (lane & 15), kf)]);
#pragma unroll
        for (int j = 0; j < FN; ++j) fb[j] = *(const FragG*)(&Bs[L::at(wn * WTN + j * 16 + (lane & 15), kf)]);
    };
    auto mma_step = [&](const FragG(&fa)[FM], const FragG(&fb)[FN]) {
#pragma unroll
        for (int u = 0; u < FG; ++u)
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int i = 0; i < FM; ++i)
                    acc[i][j] = mf::mma(FragGroup<TS>::at(fb[j], u), FragGroup<TS>::at(fa[i], u), acc[i][j]);
    };

    const int nk = g.K / BK;
#pragma unroll
    for (int p = 0; p < S - 1; ++p) issue(min(p, nk - 1), p);
    vm_wait_barrier<QMIN * (S - 2)>();   // slice 0 landed
    issue(min(S - 1, nk - 1), S - 1);
    // retire the scalar loads of the kernel arguments here: scalar loads
    // return out of order, and one still pending at the loop head would make
    // the compiler wait for all LDS reads before the first MFMA of a slice
    __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0)
    read_frags(af[0], bq[0], stage(0), 0);
    for (int kt = 0; kt < nk - 1; ++kt) {
        const TS* As = stage(kt);
#pragma unroll
        for (int t = 0; t < NSTEP; ++t) {
            if (t + 1 < NSTEP) {
                read_frags(af[(t + 1) & 1], bq[(t + 1) & 1], As, (t + 1) * KG);
            } else {
                vm_wait_barrier<QMIN * (S - 2)>();          // slice kt+1 landed
                issue(min(kt + S, nk - 1), kt % S);          // stage of slice kt is free
                read_frags(af[0], bq[0], stage(kt + 1), 0);
            }
            __builtin_amdgcn_sched_barrier(0);
            mma_step(af[t & 1], bq[t & 1]);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    {
        const TS* As = stage(nk - 1);
#pragma unroll
        for (int t = 0; t < NSTEP; ++t) {
            if (t + 1 < NSTEP) read_frags(af[(t + 1) & 1], bq[(t + 1) & 1], As, (t + 1) * KG);
            __builtin_amdgcn_sched_barrier(0);
            mma_step(af[t & 1], bq[t & 1]);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    // no direct load may still be writing LDS when the epilogue reuses it or
    // the workgroup ends
    vm_wait_barrier<0>();

    // ---- epilogue: acc[i][j][r] of lane l is C[row_i][col_j + r * ST]
    const int row0 = tile_m * BM + wm * WTM + (lane & 15);
    const int col0 = tile_n * BN + wn * WTN + mf::col0(lane);
    typedef Quad<TS, ST> Q;
    if (EPI == EPI_CELU) {
        TS* C = (TS*)g.C + (size_t)z * g.c_z;
        const TA* bias = g.bias + (size_t)s * g.bias_s + (size_t)z * g.bias_z;
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int col = col0 + j * 16;
            TA bb[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) bb[r] = bias[col + r * ST];
#pragma unroll
            for (int i = 0; i < FM; ++i) {
                TA v[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) v[r] = celu((TA)acc[i][j][r] + bb[r], g.alpha, g.inv_alpha);
                Q::st(C + (size_t)(row0 + i * 16) * g.ldc + col, v);
            }
        }
    } else if (EPI == EPI_ACC) {
        // dE/dAEV rows, in the precision's dE/dAEV storage type
        typedef typename P::TG TG;
        TG* C = (TG*)g.C + (size_t)z * g.c_z;
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int i = 0; i < FM; ++i) {
                TA v[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) v[r] = (TA)acc[i][j][r];
                Quad<TG, ST>::st(C + (size_t)(row0 + i * 16) * g.ldc + col0 + j * 16, v);
            }
    } else if (EPI == EPI_DSIG) {
        TS* C = (TS*)g.C + (size_t)z * g.c_z;
        const TS* Hr = g.Hr + (size_t)z * g.h_z;
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int i = 0; i < FM; ++i) {
                const size_t row = row0 + i * 16;
                const int col = col0 + j * 16;
                TA hh[4], v[4];
                Q::ld(Hr + row * g.ldh + col, hh);
#pragma unroll
                for (int r = 0; r < 4; ++r) v[r] = (TA)acc[i][j][r] * dcelu_h(hh[r], g.inv_alpha);
                Q::st(C + row * g.ldc + col, v);
            }
    } else if (EPI == EPI_RAW) {
        TS* C = (TS*)g.C + (size_t)z * g.c_z;
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int i = 0; i < FM; ++i) {
                TA v[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) v[r] = (TA)acc[i][j][r];
                Q::st(C + (size_t)(row0 + i * 16) * g.ldc + col0 + j * 16, v);
            }
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
            for (int i = 0; i < FM; ++i) {
                const size_t row = row0 + i * 16;
                const int col = col0 + j * 16;
                TA hh[4], ac[4], hd[4], v[4], v2[4];
                Q::ld(Hr + row * g.ldh + col, hh);
                Q::ld(X + row * g.ldx + col, ac);
                Q::ld(Tr + row * g.ldt + col, hd);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const TA d1 = dcelu_h(hh[r], g.inv_alpha);
                    const TA rho = hh[r] < TA(0) ? g.inv_alpha : TA(0);
                    v[r] = (TA)acc[i][j][r] * d1 + ac[r] * rho * hd[r];
                    v2[r] = ac[r] * d1;
                }
                Q::st(C + row * g.ldc + col, v);
                Q::st(C2 + row * g.ldc + col, v2);
            }
    } else {   // EPI_L3F
        TS* C = (TS*)g.C + (size_t)z * g.c_z;
        const TA* bias = g.bias + (size_t)s * g.bias_s + (size_t)z * g.bias_z;
        const TA* w4 = g.w4 + (size_t)s * g.w4_s + (size_t)z * g.w4_z;
        TA part[FM];
#pragma unroll
        for (int i = 0; i < FM; ++i) part[i] = 0;
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int col = col0 + j * 16;
            TA bb[4], ww[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                bb[r] = bias[col + r * ST];
                ww[r] = w4[col + r * ST];
            }
#pragma unroll
            for (int i = 0; i < FM; ++i) {
                TA v[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const TA zz = (TA)acc[i][j][r] + bb[r];
                    part[i] += ww[r] * celu(zz, g.alpha, g.inv_alpha);
                    v[r] = dcelu_z(zz, g.inv_alpha) * ww[r] * g.gscale;
                }
                Q::st(C + (size_t)(row0 + i * 16) * g.ldc + col, v);
            }
        }
        // sum over the four lane groups (same row, different columns), then
        // over the WN waves that share the row
#pragma unroll
        for (int i = 0; i < FM; ++i) {
            TA v = part[i];
            v += __shfl_xor(v, 16);
            v += __shfl_xor(v, 32);
            if (lane < 16) red[(wm * WTM + i * 16 + lane) * WN + wn] = v;
        }
        __syncthreads();
        for (int rr = tid; rr < BM; rr += 64 * NW) {
            TA v = 0;
#pragma unroll
            for (int q = 0; q < WN; ++q) v += red[rr * WN + q];
            const size_t row = (size_t)tile_m * BM + rr;
            g.epart[(row * g.n_models + z) * g.nt + tile_n] = v;
        }
    }
}

// ---------------------------------------------------------------------------
template <typename P, int BM, int BN, int WM, int WN, int S, int EPI>
static hipError_t run_gemm(GemmArgs<P> a, int Rcap, int N, int nz, hipStream_t st,
                           const Timer& tm, const char* name) {
    a.nm = Rcap / BM;
    a.nn = N / BN;
    a.nz = nz;
    if (a.K % Slice<typename P::TS>::BK != 0 || N % BN != 0 || Rcap % BM != 0) return hipErrorInvalidValue;
    const int T = a.nm * a.nn * a.nz;
    const size_t lds = GemmShape<P, BM, BN, WM, WN, S>::lds_bytes();
    auto kern = k_gemm<P, BM, BN, WM, WN, S, EPI>;
    hipError_t e = ensure_lds((const void*)kern, lds);
    if (e != hipSuccess) return e;
    tm.b(name, st);
    hipLaunchKernelGGL(kern, dim3(T), dim3(64 * WM * WN), lds, st, a);
    tm.e(name, st);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Layer-1 GEMMs in BF16 with the weight operand in registers.  On gfx950 the
// LDS returns about 64 bytes per clock per CU to ds_read_b128, which caps a
// kernel that reads both operands' fragments from LDS with 64 x 64 wave tiles
// near half the MFMA peak.  Here only the activation rows go through LDS
// (direct global->LDS loads, two stages, as in k_gemm); each wave loads its
// weight fragments straight into registers from a fragment-ordered copy of
// the weights (frag_index layout: one 1 KiB contiguous load per fragment),
// one k-step ahead.  A workgroup of 4 waves owns a 128 x 256 tile, each wave
// 128 rows x 64 columns, so LDS serves 64 FLOP per byte read and no weight
// fragment is loaded twice in a workgroup.
//
// Every k-step issues the same loads (4 fragment loads; the second step of a
// slice also 4 direct row loads), so fixed wait counts hold: a fragment is
// waited for with 8 younger loads in flight, the row slice needed next with
// 12 (S - 2) + 8.  With S = 3 the prologue issues one row slice twice (same
// data to the same LDS), which makes the first slice's count exact too.  Past
// the end the last slice and the last fragments are loaded again (L2 hits).
// The LDS fragment reads of the next k-step are interleaved with the MFMAs
// of the current one.
constexpr int kRbBM = 128, kRbBN = 256, kRbWN = 4;
constexpr int kRbRows = 128;   // bucket row tile the register-weight path runs on

template <int S, int EPI>
__global__ __launch_bounds__(256, 2) void k_l1rb(GemmArgs<PrecBF16> g) {
    typedef bf16_t TS;
    typedef float TA;
    typedef MF<TS> mf;
    typedef typename mf::Acc Acc;
    typedef typename mf::Frag Frag;
    typedef Slice<TS> L;
    constexpr int BM = kRbBM, BN = kRbBN, BK = L::BK;   // BK = 64 (two 32-deep k-steps)
    constexpr int WTN = BN / kRbWN, FM = BM / 16, FN = WTN / 16;
    constexpr int NQ = BM / 8 / kRbWN;                   // direct row loads per wave per slice
    static_assert(BK == 2 * mf::KM && NQ >= 1 && FN == 4, "tile");
    static_assert(S == 2 || S == 3, "stages");
    extern __shared__ __align__(16) char smem_raw[];
    TS* const stage0 = (TS*)smem_raw;                    // S stages of BM rows

    // tile schedule as in k_gemm (XCD-contiguous ranges, kGroupM row tiles)
    const int T = g.nm * g.nn;
    const int bid = blockIdx.x, xcd = bid & 7, slot = bid >> 3;
    const int q8 = T >> 3, r8 = T & 7;
    const int lin = xcd * q8 + (xcd < r8 ? xcd : r8) + slot;
    const int grp = lin / (kGroupM * g.nn), inside = lin % (kGroupM * g.nn);
    const int gsz = min(kGroupM, g.nm - grp * kGroupM);
    const int tile_n = inside / gsz, tile_m = grp * kGroupM + inside % gsz;

    const int rows = g.info->rows;
    if (tile_m * BM >= rows) return;
    const int s = g.tile_species[(tile_m * BM) / g.row_tile];
    if (s < 0) return;
    const int lane = threadIdx.x & 63, wn = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

    const TS* A = g.A + (size_t)tile_m * BM * g.lda;
    const int KQ = g.K / mf::KM;                         // k-steps along K
    // this wave's fragment column f (16 columns each) starts at fragment
    // (tile_n * BN / 16 + wn * FN + f, k-step 0)
    const TS* Bw = g.B + (size_t)s * g.b_s + ((size_t)(tile_n * (BN / 16) + wn * FN) * KQ * 64 + lane) * 8;

    const int ld_row = lane >> 3, ld_chunk = (lane & 7) ^ (lane >> 3);
    auto issue_rows = [&](int src, int st_) {
        TS* d = stage0 + (size_t)st_ * BM * BK;
        const int k0 = src * BK + ld_chunk * L::VE;
#pragma unroll
        for (int u = 0; u < NQ; ++u) {
            const int q = wn + kRbWN * u;
            __builtin_amdgcn_global_load_lds(NNP_GPTR(A + (size_t)(q * 8 + ld_row) * g.lda + k0),
                                             NNP_LPTR(d + q * 8 * BK), 16, 0, 0);
        }
    };
    // Fragment loads are issued as inline global_load_dwordx4: the compiler's
    // wait insertion does not follow loads whose registers are carried around
    // the loop and waits for every load in flight before the first k-step of
    // each slice.  Each use below is preceded by an explicit vm_wait that
    // leaves exactly the loads issued after it in flight, and a scheduling
    // barrier keeps the MFMAs behind that wait.  The compiler takes an inline
    // load's registers as written at issue, so nothing may read or reuse them
    // before that wait: the compiled kernels are checked for this.  (Plain
    // loads measured no faster, and the compiler then reorders them against
    // the direct row loads, which breaks the fixed wait counts.)
    Frag fb[2][FN];
    auto load_frags = [&](Frag(&b)[FN], int step) {
#pragma unroll
        for (int f = 0; f < FN; ++f)
            asm volatile("global_load_dwordx4 %0, %1, off"
                         : "=v"(b[f])
                         : "v"(Bw + ((size_t)f * KQ + step) * 64 * 8));
    };
    Frag fa[2][FM];
    auto read_rows = [&](Frag(&a)[FM], const TS* st_, int kk) {
        const int kf = kk + (lane >> 4) * mf::KL;
#pragma unroll
        for (int i = 0; i < FM; ++i) a[i] = *(const Frag*)(&st_[L::at(i * 16 + (lane & 15), kf)]);
    };
    Acc acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[i][j][r] = 0;
    auto mma = [&](const Frag(&a)[FM], const Frag(&b)[FN]) {
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int i = 0; i < FM; ++i) acc[i][j] = mf::mma(b[j], a[i], acc[i][j]);
    };
    auto stage = [&](int kt) { return stage0 + (size_t)(S == 2 ? kt & 1 : kt % S) * BM * BK; };
    // MFMAs of one k-step with the next k-step's fragment reads spread
    // among them (4 MFMAs, 1 read)
    auto mma_reads = [&](const Frag(&a)[FM], const Frag(&b)[FN], Frag(&nxt)[FM], const TS* st_, int kk) {
        read_rows(nxt, st_, kk);
        mma(a, b);
#pragma unroll
        for (int q = 0; q < FM; ++q) {
            __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);   // MFMA
            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // DS read
        }
    };

    // CELU epilogue: the accumulators start at the bias of their columns,
    // requested ahead of the first loads (the oldest loads in flight, so the
    // fixed wait counts below cover them)
    TA bb[FN][4];
    if constexpr (EPI == EPI_CELU) {
        const TA* bias = g.bias + (size_t)s * g.bias_s + tile_n * BN + wn * WTN + mf::col0(lane);
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) bb[j][r] = bias[j * 16 + r];
    }
    const int nk = g.K / BK, last = 2 * nk - 1;
#pragma unroll
    for (int p = 0; p < S - 1; ++p) issue_rows(min(p, nk - 1), p);
    load_frags(fb[0], 0);
    if (S == 3) issue_rows(min(1, nk - 1), 1);          // count padding (same rows again)
    vm_wait_barrier<S == 2 ? FN : 2 * NQ + FN>();        // rows of slice 0 landed
    issue_rows(min(S - 1, nk - 1), S - 1);
    __builtin_amdgcn_s_waitcnt(0xc07f);                  // lgkmcnt(0): kernel arguments
    read_rows(fa[0], stage(0), 0);
    if constexpr (EPI == EPI_CELU) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[i][j][r] = bb[j][r];
    }
    for (int kt = 0; kt < nk - 1; ++kt) {
        // k-step 2 kt
        load_frags(fb[1], 2 * kt + 1);
        vm_wait<NQ + FN>();                              // fragments of this step
        __builtin_amdgcn_sched_barrier(0);
        mma_reads(fa[0], fb[0], fa[1], stage(kt), mf::KM);
        __builtin_amdgcn_sched_barrier(0);
        // k-step 2 kt + 1
        load_frags(fb[0], min(2 * kt + 2, last));
        vm_wait_barrier<(NQ + 2 * FN) * (S - 2) + 2 * FN>();   // rows of slice kt+1 landed, stage of kt free
        issue_rows(min(kt + S, nk - 1), S == 2 ? kt & 1 : kt % S);
        vm_wait<NQ + FN>();
        __builtin_amdgcn_sched_barrier(0);
        mma_reads(fa[1], fb[1], fa[0], stage(kt + 1), 0);
        __builtin_amdgcn_sched_barrier(0);
    }
    {
        load_frags(fb[1], last);
        vm_wait<NQ + FN>();
        __builtin_amdgcn_sched_barrier(0);
        mma_reads(fa[0], fb[0], fa[1], stage(nk - 1), mf::KM);
        __builtin_amdgcn_sched_barrier(0);
        vm_wait_barrier<0>();                            // everything landed; no load still writes LDS
        __builtin_amdgcn_sched_barrier(0);
        mma(fa[1], fb[1]);
        __builtin_amdgcn_sched_barrier(0);
    }

    // ---- epilogue: acc[i][j][r] of lane l is C[row i*16 + l%16][col j*16 + 4 (l/16) + r]
    const int row0 = tile_m * BM + (lane & 15);
    if (EPI == EPI_CELU) {
        // lane q of a row holds 4-column pieces at 16 j + 4 q; st_strip_bf16
        // regroups them into 64-byte row segments
        TS* C = (TS*)g.C;
        TS* Cw = C + (size_t)row0 * g.ldc + tile_n * BN + wn * WTN + 8 * (lane >> 4);
#pragma unroll
        for (int i = 0; i < FM; ++i) {
            uint32_t pk[FN][2];
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                TA v[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) v[r] = celu(acc[i][j][r], g.alpha, g.inv_alpha);
                pk[j][0] = pack_bf16x2(v[0], v[1]);
                pk[j][1] = pack_bf16x2(v[2], v[3]);
            }
            st_strip_bf16(Cw + (size_t)i * 16 * g.ldc, pk, lane);
        }
    } else {   // EPI_ACC: dE/dAEV rows in bf16, 64-byte row segments as above
        TS* Cw = (TS*)g.C + (size_t)row0 * g.ldc + tile_n * BN + wn * WTN + 8 * (lane >> 4);
#pragma unroll
        for (int i = 0; i < FM; ++i) {
            uint32_t pk[FN][2];
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                pk[j][0] = pack_bf16x2(acc[i][j][0], acc[i][j][1]);
                pk[j][1] = pack_bf16x2(acc[i][j][2], acc[i][j][3]);
            }
            st_strip_bf16(Cw + (size_t)i * 16 * g.ldc, pk, lane);
        }
    }
}

static bool l1rb_fits(int Rcap, int N, int K) {
    return Rcap % kRbBM == 0 && N % kRbBN == 0 && K % Slice<bf16_t>::BK == 0 && K > 0;
}

template <int EPI>
static hipError_t run_l1rb(GemmArgs<PrecBF16> a, int Rcap, int N, int stages, hipStream_t st,
                           const Timer& tm, const char* name) {
    if (!l1rb_fits(Rcap, N, a.K) || a.B == nullptr || (stages != 2 && stages != 3)) return hipErrorInvalidValue;
    a.nm = Rcap / kRbBM;
    a.nn = N / kRbBN;
    a.nz = 1;
    const size_t lds = (size_t)stages * kRbBM * 128;
    auto kern = stages == 2 ? k_l1rb<2, EPI> : k_l1rb<3, EPI>;
    hipError_t e = ensure_lds((const void*)kern, lds);
    if (e != hipSuccess) return e;
    tm.b(name, st);
    hipLaunchKernelGGL(kern, dim3(a.nm * a.nn), dim3(64 * kRbWN), lds, st, a);
    tm.e(name, st);
    return hipGetLastError();
}

// tile shapes per row tile: BM = row tile; wide N tiles for the layer-1
// GEMMs, 64-wide for the per-model layers (widths 192 / 256); S LDS stages
template <typename P, int BM> struct Cfg;
template <typename P> struct Cfg<P, 128> {
    static constexpr int BNW = sizeof(typename P::TS) == 8 ? 64 : 128, BNN = 64, WM = 2, WN = 2, S = 3;
};
template <typename P> struct Cfg<P, 16> {
    static constexpr int BNW = 64, BNN = 64, WM = 1, WN = 4, S = 3;
};

// ---------------------------------------------------------------------------
// Fused tail of the ensemble for energies and forces: for one row tile of one
// element bucket and one model it runs layers 2 and 3, the output layer, and
// the backward through layers 3 and 2, keeping every intermediate in LDS:
//
//   H2  = celu(H1 W2^T + b2)                 -> LDS
//   z3  = H2 W3^T + b3;  e = w4 . celu(z3)   -> per-row energy partial
//   DZ3 = celu'(z3) w4 gscale                -> LDS
//   DZ2 = (DZ3 W3) celu'(H2)                 -> LDS (over H2)
//   DZ1 = (DZ2 W2) celu'(H1)                 -> HBM
//
// so HBM sees H1 once and DZ1 once per row and model.  The four waves split
// every product 1 x 4 along N: each wave needs only its own columns of the
// weights, so weight fragments go from L2 straight into registers (no LDS
// staging), while the activation operand is shared through LDS.  LDS tiles
// use the sliced layout of the GEMMs: [K / BK][rows][BK], 16-byte chunks
// XOR-swizzled by row.
template <typename TS> struct Sliced {
    static constexpr int VE = 16 / (int)sizeof(TS);
    static constexpr int BK = 8 * VE;
    __device__ static int at(int rows, int r, int k) {
        return (k / BK) * rows * BK + r * BK + ((((k % BK) / VE) ^ r) & 7) * VE + (k % VE);
    }
};

// element type of the MFMA accumulators for operand type TS
template <typename TS> using AccE = typename std::conditional<std::is_same<TS, double>::value, double, float>::type;

// acc = A rows m0 + [0, 16 FM) (LDS, sliced, BM rows, K columns) x B^T, B
// n-tiles nt0 + [0, FN) of a matrix in fragment order (one contiguous 64-lane
// load per fragment).  A stored fragment spans FragK<TS>::KM of K (one bf16
// MFMA, four FP32 or two FP64 ones); the A operand is read from LDS in the
// same grouping, one 16-byte vector per lane.  The B fragments of step t+PD
// are requested before the MFMAs of step t; the empty asm with a memory
// clobber keeps the compiler from sinking those loads next to their use, so
// PD steps of MFMAs (and the other waves) cover the L2 latency.
// K: the reduction length used; KS: the K the fragment-ordered matrix is
// stored with (its steps per n-tile); bias, if given, points at the bias of
// this lane's first column and starts the accumulators there.
template <typename TS, int BM, int FM, int FN, int K, int KS = K>
__device__ inline void tail_product(typename MF<TS>::Acc (&acc)[FM][FN], const TS* As, int m0,
                                    const TS* __restrict__ Bf, int nt0, int lane,
                                    const AccE<TS>* bias = nullptr) {
    typedef MF<TS> mf;
    typedef Sliced<TS> L;
    typedef FragGroup<TS> FGp;
    typedef typename FGp::V FragG;
    constexpr int G = FGp::G, KMS = FragK<TS>::KM, KLS = FragK<TS>::KL;
    static_assert(KMS == mf::KM * G && KLS == mf::KL * G, "stored fragment = G MFMA steps");
    // prefetch distance in stored fragments: 8 MFMA steps ahead for FP32
    // (2 x 4) and FP64 (4 x 2), 2 for bf16
    constexpr int NS = K / KMS, NSS = KS / KMS, PD = G == 2 ? 4 : 2;
    static_assert(K % KMS == 0 && K <= KS, "reduction length");
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const AccE<TS> b0 = bias ? bias[j * 16 + r * mf::kColStride] : AccE<TS>(0);
#pragma unroll
            for (int i = 0; i < FM; ++i) acc[i][j][r] = b0;
        }
    const TS* Bl = Bf + (size_t)nt0 * NSS * 64 * KLS + lane * KLS;
    FragG bq[PD + 1][FN];
#pragma unroll
    for (int t = 0; t < PD && t < NS; ++t)
#pragma unroll
        for (int j = 0; j < FN; ++j) bq[t][j] = *(const FragG*)(Bl + ((size_t)j * NSS + t) * 64 * KLS);
#pragma unroll
    for (int t = 0; t < NS; ++t) {
        if (t + PD < NS) {
#pragma unroll
            for (int j = 0; j < FN; ++j)
                bq[(t + PD) % (PD + 1)][j] = *(const FragG*)(Bl + ((size_t)j * NSS + t + PD) * 64 * KLS);
        }
        asm volatile("" ::: "memory");
        const int kf = t * KMS + (lane >> 4) * KLS;
        FragG af[FM];
#pragma unroll
        for (int i = 0; i < FM; ++i) af[i] = *(const FragG*)(&As[L::at(BM, m0 + i * 16 + (lane & 15), kf)]);
#pragma unroll
        for (int u = 0; u < G; ++u)
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int i = 0; i < FM; ++i)
                    acc[i][j] = mf::mma(FGp::at(bq[t % (PD + 1)][j], u), FGp::at(af[i], u), acc[i][j]);
    }
}

// four values of one row at columns c, c+ST, c+2ST, c+3ST of a sliced LDS tile
template <typename TS, int ST> struct LdsQuad {
    typedef typename std::conditional<sizeof(TS) == 8, double, float>::type TA;
    __device__ static void ld(const TS* T, int rows, int r, int c, TA v[4]) {
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = Store<TS>::ld(T[Sliced<TS>::at(rows, r, c + q * ST)]);
    }
    __device__ static void st(TS* T, int rows, int r, int c, const TA v[4]) {
#pragma unroll
        for (int q = 0; q < 4; ++q) T[Sliced<TS>::at(rows, r, c + q * ST)] = Store<TS>::st(v[q]);
    }
};
// contiguous case: c % 4 == 0 keeps the four values inside one 16-byte chunk
template <typename TS> struct LdsQuad<TS, 1> {
    typedef float TA;
    __device__ static void ld(const TS* T, int rows, int r, int c, TA v[4]) {
        Quad<TS, 1>::ld(T + Sliced<TS>::at(rows, r, c), v);
    }
    __device__ static void st(TS* T, int rows, int r, int c, const TA v[4]) {
        Quad<TS, 1>::st(T + Sliced<TS>::at(rows, r, c), v);
    }
};

template <typename P> struct TailArgs {
    typedef typename P::TS TS;
    typedef typename P::TA TA;
    const TS* H1; TS* DZ1; int ldh;          // [Rcap][M*H1]
    const TS* W2f; const TS* W2Tf; const TA* b2;      // fragment order
    const TS* W3f; const TS* W3Tf; const TA* b3; const TA* w4;
    TA* epart;                                // [Rcap][M]
    TA gscale, alpha, inv_alpha;
    int M;
    const int32_t* tile_species; int row_tile;
    const BucketInfo* info;
    int nm;                                   // row tiles
};

// LDS of the fused tail: H2 / DZ2 [BM][H2] at 0, DZ3 [BM][H3] after it, then
// the energy partials and the layer parameters.  The H1 tile of the first
// product spans the first two regions (it is dead once that product is
// done); for the last epilogue the H1 column quarters of waves 0-2 go to the
// DZ3 region and the fourth to the start of the DZ2 region once every wave
// is past the last product.  So the tile never needs a region of its own
// (ANI-2x widths, BF16: 51 KB, three workgroups per CU).
template <typename P, int BM, int H1, int H2, int H3>
struct TailShape {
    typedef typename P::TS TS;
    static constexpr size_t hs = (size_t)BM * H2 * sizeof(TS);
    static constexpr size_t u1 = (size_t)BM * H1 * sizeof(TS), u2 = (size_t)BM * H3 * sizeof(TS);
    static_assert(u1 <= hs + u2 && 3 * (u1 / 4) <= u2 && u1 / 4 <= hs, "H1 tile placement");
    static constexpr size_t par = sizeof(typename P::TA) * (H2 + 2 * H3);   // b2, b3, w4
    static constexpr size_t lds_bytes() { return hs + u2 + sizeof(typename P::TA) * BM * 4 + par; }
};

// H3 is the stored (padded) width of layer 3, H3L <= H3 the width the
// products use: the weights past H3L are zero padding, so layer 3 forward
// computes only H3L outputs and its backward reduces over H3L
template <typename P, int BM, int TW, int H1, int H2, int H3, int H3L = H3>
__global__ __launch_bounds__(256 * TW, 2 * TW) void k_tail(TailArgs<P> g) {
    typedef typename P::TS TS;
    typedef typename P::TA TA;
    typedef MF<TS> mf;
    typedef typename mf::Acc Acc;
    typedef Sliced<TS> L;
    constexpr int NT = 256 * TW, FM = BM / 16 / TW, ST = mf::kColStride;
    static_assert(H1 % 64 == 0 && H2 % 64 == 0 && H3 % 64 == 0 && BM % 16 == 0, "widths");
    typedef TailShape<P, BM, H1, H2, H3> Sh;
    extern __shared__ __align__(16) char smem_raw[];
    TS* H1t = (TS*)smem_raw;                             // H1 tile (first product only)
    TS* Hs = (TS*)smem_raw;                              // H2, later DZ2   [BM][H2]
    TS* Us = (TS*)(smem_raw + Sh::hs);                   // DZ3, later H1 quarters 0-2
    TA* red = (TA*)(smem_raw + Sh::hs + Sh::u2);         // [BM][4]
    TA* sb2 = red + BM * 4;            // b2 [H2], b3 [H3], w4 [H3] of this element and model
    TA* sb3 = sb2 + H2;
    TA* sw4 = sb3 + H3;

    // XCD-contiguous ranges over (model, row tile): an XCD works through
    // consecutive tiles of one model and keeps that model's weights in L2
    const int T = g.nm * g.M;
    const int bid = blockIdx.x, xcd = bid & 7, slot = bid >> 3;
    const int q8 = T >> 3, r8 = T & 7;
    const int lin = xcd * q8 + (xcd < r8 ? xcd : r8) + slot;
    const int z = lin / g.nm, tile_m = lin % g.nm;
    const int row0 = tile_m * BM;
    if (row0 >= g.info->rows) return;
    const int s = g.tile_species[row0 / g.row_tile];
    if (s < 0) return;
    const int tid = threadIdx.x, lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wn = wave & 3, m0 = (wave >> 2) * (BM / TW);   // column quarter, first row
    const size_t sz = (size_t)s * g.M + z;

    // H1 columns [c0, c0 + NC) (whole K slices) of rows [r0, r0 + NR) -> a
    // sliced LDS tile of BM rows at dst (its slice 0 = column c0), by direct
    // loads of 8 rows x one slice, dealt to waves w, w + nw, ...
    auto load_h1 = [&](TS* dst, int c0, auto nc_c, int r0, auto nr_c, int w, int nw) {
        constexpr int NC = decltype(nc_c)::value, NR = decltype(nr_c)::value;
        constexpr int NG = NR / 8, NQ = (NC / L::BK) * NG;
        static_assert(NC % L::BK == 0 && NR % 8 == 0, "whole slices and row groups");
        const TS* src0 = g.H1 + (size_t)row0 * g.ldh + (size_t)z * H1 + c0;
        const int lr = lane >> 3, lc = (lane & 7) ^ (lane >> 3);
        for (int q = w; q < NQ; q += nw) {
            const int t = q / NG, rq = r0 / 8 + q % NG;
            const TS* src = src0 + (size_t)(rq * 8 + lr) * g.ldh + t * L::BK + lc * L::VE;
            __builtin_amdgcn_global_load_lds(NNP_GPTR(src), NNP_LPTR(dst + (t * BM + rq * 8) * L::BK), 16, 0, 0);
        }
    };
    constexpr int NWV = 4 * TW, HQ = H1 / 4;   // waves; H1 columns per column quarter
    {
        load_h1(H1t, 0, std::integral_constant<int, H1>{}, 0, std::integral_constant<int, BM>{}, wave, NWV);
        // the layer parameters the epilogues read, staged beside the tile
        for (int t = tid; t < H2 + 2 * H3; t += NT) {
            const TA v = t < H2 ? g.b2[sz * H2 + t]
                                : (t < H2 + H3 ? g.b3[sz * H3 + (t - H2)] : g.w4[sz * H3 + (t - H2 - H3)]);
            sb2[t] = v;
        }
        vm_wait_barrier<0>();
    }
    const int rl = lane & 15;                 // this lane's row within each 16-row fragment
    const int cl = mf::col0(lane);            // and its first column within each 16 columns

    // ---- layer 2 forward
    {
        constexpr int FN = H2 / 64;
        Acc acc[FM][FN];
        const int n0 = wn * (H2 / 4);
        tail_product<TS, BM, FM, FN, H1>(acc, H1t, m0, g.W2f + sz * H2 * H1, n0 / 16, lane, sb2 + n0 + cl);
        __syncthreads();   // every wave is done with the H1 tile, which H2 overwrites
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int c = n0 + j * 16 + cl;
#pragma unroll
            for (int i = 0; i < FM; ++i) {
                TA v[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) v[q] = celu((TA)acc[i][j][q], g.alpha, g.inv_alpha);
                LdsQuad<TS, ST>::st(Hs, BM, m0 + i * 16 + rl, c, v);
            }
        }
    }
    __syncthreads();   // H2 complete
    // ---- layer 3 forward, output layer, dE/dz3: the H3L / 16 column tiles
    // dealt to the four waves as evenly as they go (160: 2, 3, 2, 3), each
    // wave running a product with its own static tile count
    {
        constexpr int F3 = H3L / 16, FNX = (F3 + 3) / 4;
        const int f0 = (wn * F3) / 4, fn = ((wn + 1) * F3) / 4 - f0;
        auto layer3 = [&](auto fn_c) {
            constexpr int FN = decltype(fn_c)::value;
            Acc acc[FM][FN];
            const int n0 = 16 * f0;
            tail_product<TS, BM, FM, FN, H2>(acc, Hs, m0, g.W3f + sz * H3 * H2, f0, lane, sb3 + n0 + cl);
            const TA* w4 = sw4;
            TA part[FM];
#pragma unroll
            for (int i = 0; i < FM; ++i) part[i] = 0;
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                const int c = n0 + j * 16 + cl;
                TA ww[4], wg[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    ww[q] = w4[c + q * ST];
                    wg[q] = ww[q] * g.gscale;
                }
#pragma unroll
                for (int i = 0; i < FM; ++i) {
                    TA v[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const TA zz = (TA)acc[i][j][q];
                        part[i] += ww[q] * celu(zz, g.alpha, g.inv_alpha);
                        v[q] = dcelu_z(zz, g.inv_alpha) * wg[q];
                    }
                    LdsQuad<TS, ST>::st(Us, BM, m0 + i * 16 + rl, c, v);
                }
            }
#pragma unroll
            for (int i = 0; i < FM; ++i) {
                TA v = part[i];
                v += __shfl_xor(v, 16);
                v += __shfl_xor(v, 32);
                if (lane < 16) red[(m0 + i * 16 + lane) * 4 + wn] = v;
            }
        };
        if (fn == FNX || F3 % 4 == 0) layer3(std::integral_constant<int, FNX>{});
        else layer3(std::integral_constant<int, (FNX > 1 ? FNX - 1 : 1)>{});
    }
    __syncthreads();   // DZ3 and the energy partials complete
    if (tid < BM) {
        const TA e = red[tid * 4] + red[tid * 4 + 1] + red[tid * 4 + 2] + red[tid * 4 + 3];
        g.epart[(size_t)(row0 + tid) * g.M + z] = e;
    }
    // ---- layer 3 backward: DZ2 = (DZ3 W3) celu'(H2), in place of H2 (each
    // lane reads and then overwrites only its own elements; every wave is done
    // reading H2 as an operand)
    {
        constexpr int FN = H2 / 64;
        Acc acc[FM][FN];
        const int n0 = wn * (H2 / 4);
        tail_product<TS, BM, FM, FN, H3L, H3>(acc, Us, m0, g.W3Tf + sz * H2 * H3, n0 / 16, lane);
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int c = n0 + j * 16 + cl;
#pragma unroll
            for (int i = 0; i < FM; ++i) {
                TA hh[4], v[4];
                LdsQuad<TS, ST>::ld(Hs, BM, m0 + i * 16 + rl, c, hh);
#pragma unroll
                for (int q = 0; q < 4; ++q) v[q] = (TA)acc[i][j][q] * dcelu_h(hh[q], g.inv_alpha);
                LdsQuad<TS, ST>::st(Hs, BM, m0 + i * 16 + rl, c, v);
            }
        }
    }
    __syncthreads();   // DZ2 complete
    // ---- layer 2 backward: DZ1 = (DZ2 W2) celu'(H1) -> HBM
    {
        constexpr int FN = H1 / 64;
        Acc acc[FM][FN];
        const int n0 = wn * (H1 / 4);
        TS* Out = g.DZ1 + (size_t)row0 * g.ldh + (size_t)z * H1;
        // CELU'(H1) operands of the epilogue: the H1 column quarters of waves
        // 0-2 into the region DZ3 held (every wave is past its last read of
        // DZ3), in flight during the product; whole 128-byte rows per load
        load_h1(Us, 0, std::integral_constant<int, 3 * HQ>{}, 0, std::integral_constant<int, BM>{}, wave, NWV);
        tail_product<TS, BM, FM, FN, H2>(acc, Hs, m0, g.W2Tf + sz * H1 * H2, n0 / 16, lane);
        vm_wait_barrier<0>();   // quarters 0-2 landed; every wave is done reading DZ2
        // the fourth quarter over the start of DZ2, loaded by the waves that
        // read it (each its own rows)
        if (wn == 3) {
            load_h1(Hs, 3 * HQ, std::integral_constant<int, HQ>{}, m0, std::integral_constant<int, BM / TW>{}, 0, 1);
            vm_wait<0>();
        }
        const TS* Hq = wn < 3 ? Us + (size_t)wn * BM * HQ : Hs;   // this wave's quarter (sliced, BM rows)
        TA hh[FM][FN][4];
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int i = 0; i < FM; ++i) LdsQuad<TS, ST>::ld(Hq, BM, m0 + i * 16 + rl, j * 16 + cl, hh[i][j]);
        if constexpr (std::is_same<TS, bf16_t>::value && FN == 4) {
#pragma unroll
            for (int i = 0; i < FM; ++i) {
                uint32_t pk[FN][2];
#pragma unroll
                for (int j = 0; j < FN; ++j) {
                    TA v[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) v[q] = (TA)acc[i][j][q] * dcelu_h(hh[i][j][q], g.inv_alpha);
                    pk[j][0] = pack_bf16x2(v[0], v[1]);
                    pk[j][1] = pack_bf16x2(v[2], v[3]);
                }
                st_strip_bf16(Out + (size_t)(m0 + i * 16 + rl) * g.ldh + n0 + 2 * cl, pk, lane);
            }
        } else {
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                const int c = n0 + j * 16 + cl;
#pragma unroll
                for (int i = 0; i < FM; ++i) {
                    TA v[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) v[q] = (TA)acc[i][j][q] * dcelu_h(hh[i][j][q], g.inv_alpha);
                    Quad<TS, ST>::st(Out + (size_t)(m0 + i * 16 + rl) * g.ldh + c, v);
                }
            }
        }
    }
}

// the fused tail is compiled for the ANI-2x hidden widths (256, 192, 160
// padded to 192); other widths take the per-layer GEMMs
constexpr int kTailH1 = 256, kTailH2 = 192, kTailH3 = 192;

template <typename P, int BM, int TW, int H3L = kTailH3>
static hipError_t run_tail(const Shape& sh, const DevWeights<P>& wt, Work<P>& w, hipStream_t st,
                           const Timer& tm) {
    typedef typename P::TA TA;
    TailArgs<P> a{};
    a.H1 = w.H1; a.DZ1 = w.DZ1; a.ldh = sh.M * sh.H1;
    a.W2f = wt.W2f; a.W2Tf = wt.W2Tf; a.b2 = wt.b2;
    a.W3f = wt.W3f; a.W3Tf = wt.W3Tf; a.b3 = wt.b3; a.w4 = wt.w4;
    a.epart = w.Epart;
    a.gscale = (TA)(sh.energy_scale / sh.M);
    a.alpha = (TA)sh.celu_alpha;
    a.inv_alpha = (TA)(1.0 / sh.celu_alpha);
    a.M = sh.M;
    a.tile_species = w.tile_species; a.row_tile = sh.row_tile;
    a.info = w.info;
    a.nm = sh.Rcap / BM;
    const int T = a.nm * sh.M;
    const size_t lds = TailShape<P, BM, kTailH1, kTailH2, kTailH3>::lds_bytes();
    auto kern = k_tail<P, BM, TW, kTailH1, kTailH2, kTailH3, H3L>;
    hipError_t e = ensure_lds((const void*)kern, lds);
    if (e != hipSuccess) return e;
    tm.b("mlp_tail", st);
    hipLaunchKernelGGL(kern, dim3(T), dim3(256 * TW), lds, st, a);
    tm.e("mlp_tail", st);
    return hipGetLastError();
}

bool mlp_fused_supported(int H1, int H2, int H3) {
    return H1 == kTailH1 && H2 == kTailH2 && H3 == kTailH3;
}

// tail row tile per precision: equal LDS bytes (H1 tile of 32 KiB)
template <typename P> struct TailBM { static constexpr int v = 128 / (int)sizeof(typename P::TS); };

// the wide layer-1 GEMMs: LDS stages and waves per workgroup from the knobs
// (8 waves split the 128 x 128 tile 2 x 4, for 128-row buckets only)
template <typename P, int BM, int EPI>
static hipError_t run_l1(GemmArgs<P> a, const Shape& sh, int N, hipStream_t st, const Timer& tm,
                         const char* name) {
    typedef Cfg<P, BM> C;
    const int R = sh.Rcap;
    // 8 waves (2 x 4 of 64 x 32) for the forward GEMM when the knob says so;
    // the backward GEMM measured better on 4
    if constexpr (BM == 128 && C::BNW == 128 && EPI == EPI_CELU) {
        if (sh.gemm_waves == 8)
            return sh.gemm_stages == 2 ? run_gemm<P, BM, C::BNW, 2, 4, 2, EPI>(a, R, N, 1, st, tm, name)
                                       : run_gemm<P, BM, C::BNW, 2, 4, 3, EPI>(a, R, N, 1, st, tm, name);
    }
    // 16-row tiles (small batches) stream the weights through a deeper pipeline:
    // few workgroups, so each keeps more loads in flight (BF16 6 stages; FP32
    // and FP64, whose slices hold half or a quarter of the K, measured best at 4)
    if constexpr (BM == 16) {
        constexpr int S16 = sizeof(typename P::TS) == 2 ? 6 : 4;
        return run_gemm<P, BM, C::BNW, C::WM, C::WN, S16, EPI>(a, R, N, 1, st, tm, name);
    }
    return sh.gemm_stages == 2 ? run_gemm<P, BM, C::BNW, C::WM, C::WN, 2, EPI>(a, R, N, 1, st, tm, name)
                               : run_gemm<P, BM, C::BNW, C::WM, C::WN, 3, EPI>(a, R, N, 1, st, tm, name);
}

// L1b: dG = DZ1cat W1cat (models summed along K)
template <typename P, int BM>
static hipError_t mlp_l1_bwd(const Shape& sh, const DevWeights<P>& wt, Work<P>& w,
                             const GemmArgs<P>& base, hipStream_t st, const Timer& tm) {
    typedef Cfg<P, BM> C;
    const int M = sh.M, H1 = sh.H1, Dp = sh.Dp, R = sh.Rcap;
    GemmArgs<P> a = base;
    a.A = w.DZ1; a.lda = M * H1; a.a_z = 0;
    a.B = wt.W1T; a.ldb = M * H1; a.b_s = (long)Dp * M * H1; a.b_z = 0;
    a.C = w.dG; a.ldc = Dp; a.c_z = 0;
    a.K = M * H1;
    if constexpr (std::is_same<P, PrecBF16>::value && BM == kRbRows) {
        if (sh.l1_path == 2) {
            a.B = wt.W1Tf;
            return run_l1rb<EPI_ACC>(a, R, Dp, sh.gemm_stages, st, tm, "mlp_l1_bwd");
        }
    }
    if (Dp % C::BNW == 0) return run_l1<P, BM, EPI_ACC>(a, sh, Dp, st, tm, "mlp_l1_bwd");
    return run_gemm<P, BM, C::BNN, C::WM, C::WN, C::S, EPI_ACC>(a, R, Dp, 1, st, tm, "mlp_l1_bwd");
}

template <typename P, int BM>
static hipError_t mlp_all(const Shape& sh, const DevWeights<P>& wt, Work<P>& w, hipStream_t st,
                          const Timer& tm) {
    typedef typename P::TA TA;
    typedef Cfg<P, BM> C;
    const int M = sh.M, H1 = sh.H1, H2 = sh.H2, H3 = sh.H3, Dp = sh.Dp;
    hipError_t e = hipSuccess;
    GemmArgs<P> base{};
    base.tile_species = w.tile_species;
    base.row_tile = sh.row_tile;
    base.info = w.info;
    base.alpha = (TA)sh.celu_alpha;
    base.inv_alpha = (TA)(1.0 / sh.celu_alpha);
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
    bool l1_done = false;
    if constexpr (std::is_same<P, PrecBF16>::value && BM == kRbRows) {
        if (sh.l1_path == 2) {
            a.B = wt.W1f;
            e = run_l1rb<EPI_CELU>(a, R, M * H1, sh.gemm_stages, st, tm, "mlp_l1_fwd");
            l1_done = true;
        }
    }
    if (l1_done)
        ;
    else if ((M * H1) % C::BNW == 0)
        e = run_l1<P, BM, EPI_CELU>(a, sh, M * H1, st, tm, "mlp_l1_fwd");
    else
        e = run_gemm<P, BM, C::BNN, C::WM, C::WN, C::S, EPI_CELU>(a, R, M * H1, 1, st, tm, "mlp_l1_fwd");
    if (e) return e;
    if (sh.mlp_fused) {
        if (!mlp_fused_supported(H1, H2, H3)) return hipErrorInvalidValue;
        // fused layers 2-3 forward and backward
        w.epart_nt = 1;
        constexpr int TB = TailBM<P>::v, TH = TB / 2 >= 16 ? TB / 2 : 16;
        // layer 3 of at most 160 outputs (ANI-2x): products over the 160 real
        // columns, not the 192 the storage is padded to
        const bool n160 = sh.h3_used <= 160;
        if (BM == 16) e = n160 ? run_tail<P, 16, 1, 160>(sh, wt, w, st, tm) : run_tail<P, 16, 1>(sh, wt, w, st, tm);
        else if (sh.tail_tile == 2)
            e = n160 ? run_tail<P, TH, 1, 160>(sh, wt, w, st, tm) : run_tail<P, TH, 1>(sh, wt, w, st, tm);
        else if (sh.tail_tile == 3 && TB >= 32)
            e = n160 ? run_tail<P, TB, TB >= 32 ? 2 : 1, 160>(sh, wt, w, st, tm)
                     : run_tail<P, TB, TB >= 32 ? 2 : 1>(sh, wt, w, st, tm);
        else e = n160 ? run_tail<P, TB, 1, 160>(sh, wt, w, st, tm) : run_tail<P, TB, 1>(sh, wt, w, st, tm);
        if (e) return e;
        return mlp_l1_bwd<P, BM>(sh, wt, w, base, st, tm);
    }
    w.epart_nt = H3 / 64;
    // L2f
    a = base;
    a.A = w.H1; a.lda = M * H1; a.a_z = H1;
    a.B = wt.W2; a.ldb = H1; a.b_s = (long)M * H2 * H1; a.b_z = (long)H2 * H1;
    a.bias = wt.b2; a.bias_s = (long)M * H2; a.bias_z = H2;
    a.C = w.H2; a.ldc = M * H2; a.c_z = H2;
    a.K = H1;
    if ((e = run_gemm<P, BM, C::BNN, C::WM, C::WN, C::S, EPI_CELU>(a, R, H2, M, st, tm, "mlp_l2_fwd")))
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
    if ((e = run_gemm<P, BM, 64, C::WM, C::WN, C::S, EPI_L3F>(a, R, H3, M, st, tm, "mlp_l3_fwd")))
        return e;
    // L3b
    a = base;
    a.A = w.DZ3; a.lda = M * H3; a.a_z = H3;
    a.B = wt.W3T; a.ldb = H3; a.b_s = (long)M * H2 * H3; a.b_z = (long)H2 * H3;
    a.Hr = w.H2; a.ldh = M * H2; a.h_z = H2;
    a.C = w.DZ2; a.ldc = M * H2; a.c_z = H2;
    a.K = H3;
    if ((e = run_gemm<P, BM, C::BNN, C::WM, C::WN, C::S, EPI_DSIG>(a, R, H2, M, st, tm, "mlp_l3_bwd")))
        return e;
    // L2b
    a = base;
    a.A = w.DZ2; a.lda = M * H2; a.a_z = H2;
    a.B = wt.W2T; a.ldb = H2; a.b_s = (long)M * H1 * H2; a.b_z = (long)H1 * H2;
    a.Hr = w.H1; a.ldh = M * H1; a.h_z = H1;
    a.C = w.DZ1; a.ldc = M * H1; a.c_z = H1;
    a.K = H2;
    if (H1 % C::BNW == 0)
        e = run_gemm<P, BM, C::BNW, C::WM, C::WN, C::S, EPI_DSIG>(a, R, H1, M, st, tm, "mlp_l2_bwd");
    else
        e = run_gemm<P, BM, C::BNN, C::WM, C::WN, C::S, EPI_DSIG>(a, R, H1, M, st, tm, "mlp_l2_bwd");
    if (e) return e;
    return mlp_l1_bwd<P, BM>(sh, wt, w, base, st, tm);
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
    base.inv_alpha = (TA)(1.0 / sh.celu_alpha);
    base.gscale = (TA)(sh.energy_scale / M);
    base.n_models = M;
    base.nt = H3 / 64;
    GemmArgs<P> a;
#define NNP_RUN(EPI, N, NZ, NAME)                                                               \
    if ((e = run_gemm<P, BM, BN, C::WM, C::WN, C::S, EPI>(a, R, N, NZ, st, tm, NAME))) return e;

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
    base.inv_alpha = (TA)(1.0 / sh.celu_alpha);
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

// dG = DZ1cat W1cat alone (the AEV-row adjoint of whatever DZ1 holds)
template <typename P>
hipError_t launch_l1_bwd(const Shape& sh, const DevWeights<P>& wt, Work<P>& w, hipStream_t st,
                         const Timer& tm) {
    GemmArgs<P> base{};
    base.tile_species = w.tile_species;
    base.row_tile = sh.row_tile;
    base.info = w.info;
    base.n_models = sh.M;
    if (sh.row_tile == 128) return mlp_l1_bwd<P, 128>(sh, wt, w, base, st, tm);
    if (sh.row_tile == 16) return mlp_l1_bwd<P, 16>(sh, wt, w, base, st, tm);
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
                                                TrainWork<P>&, hipStream_t, const Timer&);       \
    template hipError_t launch_l1_bwd<P>(const Shape&, const DevWeights<P>&, Work<P>&,         \
                                         hipStream_t, const Timer&);
NNP_TRAIN_INST(PrecF64)
NNP_TRAIN_INST(PrecF32)

template hipError_t launch_mlp<PrecF64>(const Shape&, const DevWeights<PrecF64>&, Work<PrecF64>&,
                                        hipStream_t, const Timer&);
template hipError_t launch_mlp<PrecF32>(const Shape&, const DevWeights<PrecF32>&, Work<PrecF32>&,
                                        hipStream_t, const Timer&);
template hipError_t launch_mlp<PrecBF16>(const Shape&, const DevWeights<PrecBF16>&,
                                         Work<PrecBF16>&, hipStream_t, const Timer&);

}  // namespace nnp
