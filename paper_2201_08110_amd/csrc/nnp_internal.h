// nnp_internal.h -- shared declarations of the HIP library (kernels + runtime).
//
// Data flow of one evaluation (all device-resident, one stream):
//   prep        element counts, padded per-element row buckets, atom->row map
//   neighbours  per-atom neighbour lists inside each molecule (angular first)
//   aev         per-atom AEV rows written in bucket order (GEMM operand type)
//   mlp         six GEMMs per element bucket, all ensemble members at once:
//                 layer-1 forward (models concatenated along N), layers 2-3
//                 forward (per model), layer-3 backward, layer-2 backward,
//                 layer-1 backward (models summed along K) -> dE/dAEV;
//                 activations are stored after CELU and CELU' is recovered
//                 from them
//   forces      AEV backward contracted with dE/dAEV, scattered to atoms
//   energy      per-molecule FP64 sum of the atomic energies
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <utility>

namespace nnp {

// ---------------------------------------------------------------------------
// bf16 storage: raw 16-bit patterns, round-to-nearest-even from float.
typedef uint16_t bf16_t;

__host__ __device__ inline bf16_t f2bf(float f) {
    uint32_t u;
    __builtin_memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (bf16_t)((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (bf16_t)(u >> 16);
}
__host__ __device__ inline float bf2f(bf16_t h) {
    uint32_t u = ((uint32_t)h) << 16;
    float f;
    __builtin_memcpy(&f, &u, 4);
    return f;
}

// device conversion of two floats to packed bf16 (low half = a): the
// hardware's round-to-nearest-even conversion, the same rounding as f2bf
typedef float nnp_f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 nnp_bf16x2 __attribute__((ext_vector_type(2)));
__device__ inline uint32_t pack_bf16x2(float a, float b) {
    const nnp_f32x2 v = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, nnp_bf16x2));
}

// conversion between storage type S and arithmetic type A
template <typename S> struct Store;
template <> struct Store<float> {
    __device__ static float ld(float v) { return v; }
    __device__ static float st(float v) { return v; }
};
template <> struct Store<double> {
    __device__ static double ld(double v) { return v; }
    __device__ static double st(double v) { return v; }
};
template <> struct Store<bf16_t> {
    __device__ static float ld(bf16_t v) { return bf2f(v); }
    __device__ static bf16_t st(float v) { return (bf16_t)(pack_bf16x2(v, 0.f) & 0xffffu); }
};

// ---------------------------------------------------------------------------
// Precision modes: T = featuriser / force arithmetic, TS = GEMM operand
// storage, TA = GEMM accumulator and epilogue arithmetic, TG = storage of the
// dE/dAEV rows the layer-1 backward hands to the force kernel (BF16 handles
// keep them in bf16 like every other operand between their kernels).
struct PrecF64  { typedef double T; typedef double TS; typedef double TA; typedef double TG; };
struct PrecF32  { typedef float  T; typedef float  TS; typedef float  TA; typedef float  TG; };
struct PrecBF16 { typedef float  T; typedef bf16_t TS; typedef float  TA; typedef bf16_t TG; };

constexpr int kMaxSpecies = 8;
constexpr int kNR = 16;          // radial shifts supported by the kernels
constexpr int kNAZ = 32;         // angular (distance x angle) shifts supported
constexpr int kMaxNA = 16;       // angular-distance shifts (<= 32 / 1)
constexpr int kMaxAtomsPerMol = 1024;
constexpr int kPrepBlock = 1024;   // atoms per block of the bucketing kernels
constexpr int kMaxNeighbours = 192;
constexpr int kZLut = 128;       // atomic numbers a handle's element table may hold: 1..127

// featuriser constants, passed by value to the kernels
template <typename T> struct AevConst {
    int S, nR, nA, nZ, D, Dp;
    T rcr, rca, rcr2, rca2, eta_r, eta_a, zeta, angle_scale, radial_pref;
    T pi_rcr, pi_rca;                 // pi / Rc
    T shf_r[kNR];
    T shf_a[kMaxNA];
    T cos_z[kNAZ], sin_z[kNAZ];
};

// device error flag bits
enum : int32_t { FLAG_SPECIES = 1, FLAG_CAPACITY = 2 };

// bucket bookkeeping written by the prep kernel
struct BucketInfo {
    int32_t rows;                      // padded rows in use (multiple of the row tile)
    int32_t off[kMaxSpecies + 1];      // padded bucket starts
    int32_t count[kMaxSpecies];        // atoms per element
};

// ---------------------------------------------------------------------------
// workspace views used by the launchers
template <typename P> struct Work {
    typedef typename P::T T;
    typedef typename P::TS TS;
    typedef typename P::TA TA;
    int32_t* row_of_atom;   // [A]
    int32_t* atom_of_row;   // [Rcap]   -1 for padding rows
    int32_t* mol_of_atom;   // [A]
    int32_t* tile_species;  // [Rcap / row_tile]
    int32_t* blk;           // [2][n_blocks][kMaxSpecies]  per-block counts / bases
    BucketInfo* info;
    int32_t* flag;
    const int8_t* zlut;     // [kZLut] element index of each atomic number (-1: none), or null
                            // when batches carry element indices
    int32_t* sp;            // [A]  element indices mapped from atomic numbers (zlut != null)
    uint16_t* nbr;          // [A][cap_nbr]  local indices, angular (r < rca) first
    int32_t* nbr_cnt;       // [A]  n_ang | (n_all << 16)
    TS* G;                  // [Rcap][Dp]
    TS* H1;                 // [Rcap][M*H1]  layer-1 activations CELU(z1)
    TS* H2;                 // [Rcap][M*H2]  layer-2 activations CELU(z2)
    TS* DZ3;                // [Rcap][M*H3]
    TS* DZ2;                // [Rcap][M*H2]
    TS* DZ1;                // [Rcap][M*H1]
    TA* Epart;              // [Rcap][M][epart_nt]  per-row energy partials
    int epart_nt;           // partials per row and model (set by launch_mlp)
    typename P::TG* dG;     // [Rcap][Dp]
    unsigned long long* Fq; // [A][3]  fixed-point force sums (2^32 units, two's complement)
    int32_t* moff;          // [max_mols+1]  offsets padded to the launch bound (device counts)
    int32_t* dcnt;          // [2]  the batch's molecule and atom counts (device counts)
};

// extra workspace of the training backward (allocated on its first call)
template <typename P> struct TrainWork {
    typedef typename P::TS TS;
    TS* GD;     // [Rcap][Dp]     AEV tangent along the force cotangent
    TS* H3;     // [Rcap][M*H3]   layer-3 activations
    TS* TH1;    // [Rcap][M*H1]   tangent activations
    TS* TH2;    // [Rcap][M*H2]
    TS* TH3;    // [Rcap][M*H3]
    TS* ZDB1;   // [Rcap][M*H1]   adjoints of the tangent pre-activations
    TS* ZDB2;   // [Rcap][M*H2]
    TS* ZDB3;   // [Rcap][M*H3]
    TS* TMP;    // [Rcap][M*max(H1,H2)]
};

// host-computed layout of one network inside the packed parameter array
struct NetLayout {
    int o1, o2, o3, D;                 // unpadded widths
    long offW1, offb1, offW2, offb2, offW3, offb3, offw4, offb4, net;
};

// Stored MFMA operand fragment of the network kernels: KM = K extent of one
// fragment, KL = consecutive K elements one lane holds, 16 bytes in every
// precision.  Lane l holds row l % 16, K elements (l / 16) KL ... + KL - 1.
// A bf16 fragment (32, 8) feeds one 16x16x32 MFMA; an f32 (16, 4) or f64
// (8, 2) fragment feeds four or two 16x16x4 MFMAs, step j taking element j
// of every lane (so step j reduces over k = j, KL + j, 2 KL + j, 3 KL + j).
template <typename TS> struct FragK { static constexpr int KM = 16, KL = 4; };
template <> struct FragK<double> { static constexpr int KM = 8, KL = 2; };
template <> struct FragK<bf16_t> { static constexpr int KM = 32, KL = 8; };

// A [N][K] row-major matrix in fragment order: fragment (n-tile t, k-step q)
// occupies 64 KL consecutive elements, lane l's KL elements at l KL, so one
// wave reads a fragment with one contiguous load.
template <typename TS> __host__ __device__ inline size_t frag_index(int n, int k, int K) {
    constexpr int KM = FragK<TS>::KM, KL = FragK<TS>::KL;
    const int t = n / 16, r = n % 16, q = k / KM, kk = k % KM;
    const int lane = r + 16 * (kk / KL);
    return (((size_t)t * (K / KM) + q) * 64 + lane) * KL + kk % KL;
}

// packed device weights (per precision)
template <typename P> struct DevWeights {
    typedef typename P::TS TS;
    typedef typename P::TA TA;
    TS* W1;   TS* W1T;   TA* b1;   // [S][M*H1][Dp], [S][Dp][M*H1], [S][M*H1]
    TS* W2;   TS* W2T;   TA* b2;   // [S][M][H2][H1], [S][M][H1][H2], [S][M][H2]
    TS* W3;   TS* W3T;   TA* b3;   // [S][M][H3][H2], [S][M][H2][H3], [S][M][H3]
    TA* w4;   TA* b4;              // [S][M][H3], [S][M]
    // the fused layers 2-3 kernel's operands in fragment order (per element
    // and model: W2 [H2][H1], W3 [H3][H2], W3^T [H2][H3], W2^T [H1][H2])
    TS* W2f;  TS* W3f;  TS* W3Tf;  TS* W2Tf;
    // the layer-1 GEMMs' weight operands in fragment order (BF16 only, per
    // element: W1cat [M*H1][Dp] and W1cat^T [Dp][M*H1]; null otherwise)
    TS* W1f;  TS* W1Tf;
    double* sae;                   // [S] FP64 (already multiplied by energy_scale)
};

// where each packed parameter goes: the uniform packed layout (per-element
// networks already mapped into it) and the padded device widths
struct ParamPack {
    int S, M, D, Dp, H1, H2, H3;   // device widths (hidden widths padded to 64)
    int o1, o2;                    // widths of the packed layout's first two hidden layers
    long net, offb1, offW2, offb2, offW3, offb3, offw4, offb4;
};
template <typename P, typename TSRC>
hipError_t launch_set_params(int64_t n, const TSRC* src, const int32_t* map, const ParamPack& pk,
                             const DevWeights<P>& dw, hipStream_t st);

struct Shape {
    int S, M, D, Dp, H1, H2, H3;       // H* padded to multiples of 64
    int A, B;                          // atoms, molecules of this call
    int Rcap;                          // capacity rows
    int row_tile;                      // bucket padding = GEMM row tile
    int cap_nbr;
    int max_apm;
    double energy_scale;
    double celu_alpha;
    // kernel variants in effect (resolved tunable knobs)
    int mlp_fused;                     // 1: fused layers 2-3 kernel, 0: per-layer GEMMs
    int gemm_stages;                   // LDS stages of the layer-1 GEMMs (2 or 3)
    int gemm_waves;                    // waves per workgroup of the layer-1 forward GEMM (4 or 8)
    int l1_path;                       // layer-1 GEMMs: 1 = both operands through LDS, 2 = weights in registers
    int cell_min;                      // molecules above this many atoms use cutoff cells
    int tail_tile;                     // fused kernel tile variant (1, 2 or 3)
    int chunk;                         // central atoms per featuriser / force workgroup (4, 8, 16)
    int force_fixed;                   // 1: forces summed in 64-bit fixed point (bitwise reproducible)
    int force_path;                    // force kernel: 1 dE/dAEV row staged in LDS, 2 read from global
    int h3_used;                       // layer-3 width before padding (the widest element network's)
    int dev_counts;                    // 1: A and B are launch bounds; the counts are in Work::dcnt
    int sub;                           // 1: one part of a pipelined evaluation (atoms need not start at 0)
    int pipeline;                      // 2: large batches evaluated as two pipelined parts on two streams
};
hipError_t launch_stage_batch(int B, int A, const int32_t* counts, const int32_t* mol_off, int32_t* moff,
                              int32_t* dcnt, int32_t* flag, hipStream_t st);

// kernel timing hook (runtime-side); launchers call these around launches
struct Timer {
    void (*begin)(void* ctx, const char* name, hipStream_t s);
    void (*end)(void* ctx, const char* name, hipStream_t s);
    void* ctx;
    void b(const char* n, hipStream_t s) const { if (begin) begin(ctx, n, s); }
    void e(const char* n, hipStream_t s) const { if (end) end(ctx, n, s); }
};

// Raise a kernel's dynamic-LDS limit once per (kernel, device): later calls
// (including those recorded into a HIP graph) do no host-side work.
inline hipError_t ensure_lds(const void* kern, size_t bytes) {
    static std::mutex mu;
    static std::map<std::pair<const void*, int>, size_t> done;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = -1;
    std::lock_guard<std::mutex> g(mu);
    auto key = std::make_pair(kern, dev);
    auto it = done.find(key);
    if (it != done.end() && it->second >= bytes) return hipSuccess;
    hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e == hipSuccess) done[key] = bytes;
    return e;
}

// NNP-MM coupling (fixed at creation of a coupling handle)
// MM atoms per MM-side coupling workgroup (four lanes each): the size of the
// per-workgroup energy partials the handle allocates
constexpr int kCoupleMmPerBlock = 64;

struct CouplingShape {
    double coulomb_k;   // 1 / (4 pi eps0) in the caller's units
    double cutoff;      // 0: every pair
    int max_nnp, max_mm;
    int chunk;          // MM atoms per workgroup of the NNP-side force kernel
};
// Bytes of the per-device static scratch behind nnp_coupling_eval_noalloc
// and its device address on the current device (looked up once per device).
constexpr size_t kCoupleScratchBytes = (size_t)8 << 20;
hipError_t coupling_scratch(void** ptr);

template <typename T>
hipError_t launch_coupling(const CouplingShape& cs, int n_nnp, const T* x_nnp, const T* par_nnp,
                           int n_mm, const T* x_mm, const T* par_mm, double* E, T* F_nnp, T* F_mm,
                           double* e_part, T* f_part, bool accumulate, hipStream_t st);

// launchers (explicitly instantiated for PrecF64 / PrecF32 / PrecBF16)
template <typename P>
hipError_t launch_prep(const Shape& sh, const int32_t* mol_off, const int32_t* species,
                       Work<P>& w, hipStream_t st, const Timer& tm);
template <typename P>
hipError_t launch_neighbours(const Shape& sh, const AevConst<typename P::T>& c,
                             const int32_t* mol_off, const int32_t* species,
                             const typename P::T* x, typename P::T* F, bool accumulate, Work<P>& w,
                             hipStream_t st, const Timer& tm);
// The featuriser finding its own neighbour lists (nbr null: it reads them):
// cutoffs, the force accumulators it clears, and where the lists go
// (bucketing, for batches of at most kPrepBlock atoms and molecules: the
// bucketing kernel's outputs, written by the featuriser instead; info null:
// the bucketing kernel has run)
struct BucketFuse {
    const int8_t* zlut = nullptr;      // atomic number -> element, or null
    int32_t* sp_out = nullptr;         // element indices (zlut != null)
    int32_t* mol_of_atom = nullptr;
    int32_t* row_of_atom = nullptr;
    int32_t* atom_of_row = nullptr;
    int32_t* tile_species = nullptr;
    BucketInfo* info = nullptr;
    const int32_t* dA = nullptr;       // device atom count, or null
    int B = 0, row_tile = 16, Rcap = 0, sub = 0;
};
template <typename T> struct NbrFuse {
    T rca2 = 0, rcr2 = 0;
    T* F = nullptr;
    unsigned long long* Fq = nullptr;
    uint16_t* nbr = nullptr;
    int32_t* cnt = nullptr;
    int32_t* flag = nullptr;
    BucketFuse bk;
};
template <typename P>
hipError_t launch_aev(const Shape& sh, const AevConst<typename P::T>& c, const int32_t* mol_off,
                      const int32_t* species, const typename P::T* x, Work<P>& w,
                      typename P::T* aev_out, hipStream_t st, const Timer& tm,
                      const NbrFuse<typename P::T>& nf = NbrFuse<typename P::T>());
// bucketing, neighbour lists and AEV rows of an evaluation (species as the
// batch gives them: atomic numbers on handles with an element table)
template <typename P>
hipError_t launch_prep_features(const Shape& sh, const AevConst<typename P::T>& c, const int32_t* mol_off,
                                const int32_t* species, const typename P::T* x, typename P::T* F,
                                bool accumulate, Work<P>& w, typename P::T* aev_out, hipStream_t st,
                                const Timer& tm);
template <typename P>
hipError_t launch_features(const Shape& sh, const AevConst<typename P::T>& c, const int32_t* mol_off,
                           const int32_t* species, const typename P::T* x, typename P::T* F,
                           bool accumulate, Work<P>& w, typename P::T* aev_out, hipStream_t st,
                           const Timer& tm);
// hidden widths (padded) the fused layers 2-3 kernel is compiled for
bool mlp_fused_supported(int H1, int H2, int H3);

template <typename P>
hipError_t launch_mlp(const Shape& sh, const DevWeights<P>& wt, Work<P>& w, hipStream_t st,
                      const Timer& tm);
template <typename P>
hipError_t launch_aev_jvp(const Shape& sh, const AevConst<typename P::T>& c,
                          const int32_t* mol_off, const int32_t* species,
                          const typename P::T* x, const typename P::T* v, Work<P>& w,
                          typename P::TS* Gd, hipStream_t st, const Timer& tm);
// Per-molecule energies computed inside the force kernel (E null: none)
template <typename P> struct EnergyArgs {
    double* E = nullptr;
    const typename P::TA* Epart = nullptr;
    const typename P::TA* b4 = nullptr;
    const double* sae = nullptr;
    double scale = 0.0;
    int M = 0, NT = 0, B = 0, accumulate = 0;
    const int32_t* dcnt = nullptr;
};
template <typename P>
hipError_t launch_forces(const Shape& sh, const AevConst<typename P::T>& c,
                         const int32_t* mol_off, const int32_t* species, const typename P::T* x,
                         Work<P>& w, typename P::T* F, hipStream_t st, const Timer& tm,
                         const EnergyArgs<P>& ea = EnergyArgs<P>());
template <typename P>
EnergyArgs<P> energy_args(const Shape& sh, const DevWeights<P>& wt, Work<P>& w, double* E, bool accumulate);
template <typename P>
hipError_t launch_train_mlp(const Shape& sh, const DevWeights<P>& wt, Work<P>& w,
                            TrainWork<P>& tw, const int32_t* mol_of_atom, const double* grad_E,
                            bool has_gF, hipStream_t st, const Timer& tm);
template <typename P>
hipError_t launch_train_mlp_rev(const Shape& sh, const DevWeights<P>& wt, Work<P>& w,
                                TrainWork<P>& tw, hipStream_t st, const Timer& tm);
template <typename P>
hipError_t launch_train_rev3(const Shape& sh, const DevWeights<P>& wt, Work<P>& w,
                             TrainWork<P>& tw, const int32_t* mol_of_atom, const double* grad_E,
                             bool has_gF, hipStream_t st, const Timer& tm);
template <typename P>
hipError_t launch_train_grads(const Shape& sh, const NetLayout& nl, Work<P>& w, TrainWork<P>& tw,
                              const int32_t* mol_of_atom, const double* grad_E, bool has_gF,
                              typename P::TA* grad_params, hipStream_t st, const Timer& tm);
template <typename P>
hipError_t launch_fill(typename P::TS* p, size_t n, hipStream_t st);
template <typename P>
hipError_t launch_l1_bwd(const Shape& sh, const DevWeights<P>& wt, Work<P>& w, hipStream_t st,
                         const Timer& tm);
template <typename P>
hipError_t launch_forces_tan(const Shape& sh, const AevConst<typename P::T>& c,
                             const int32_t* mol_off, const int32_t* species, const typename P::T* x,
                             const typename P::T* v, Work<P>& w, typename P::T* Tout, hipStream_t st,
                             const Timer& tm);
template <typename T> hipError_t launch_sub(size_t n, const T* xv, T* y, hipStream_t st);
template <typename TA>
hipError_t launch_gather(int64_t n, const int32_t* map, const TA* src, TA* dst, hipStream_t st);
template <typename P>
hipError_t launch_grad_coords(int A, const int32_t* mol_of_atom, const double* grad_E,
                              const typename P::T* F, typename P::T* gx, hipStream_t st);
template <typename P>
hipError_t launch_energy(const Shape& sh, const DevWeights<P>& wt, const int32_t* mol_off,
                         const int32_t* species, Work<P>& w, double* E, typename P::T* F,
                         bool accumulate, hipStream_t st, const Timer& tm);

}  // namespace nnp
