// nnp_coupling.hip -- the NNP-MM coupling term of an NNP/MM step.
//
// Mechanical embedding (Methods, Eq. 4): every NNP atom i interacts with
// every MM atom j through a Coulomb term k q_i q_j / r and a 12-6
// Lennard-Jones term 4 eps_ij ((sigma_ij/r)^12 - (sigma_ij/r)^6), with
// Lorentz-Berthelot pair parameters sigma_ij = (sigma_i + sigma_j)/2,
// eps_ij = sqrt(eps_i eps_j) and an optional plain cutoff.  Forces act on both
// sides.  Both force sums are formed without atomics and in a fixed order:
//
//   MM side       four lanes per MM atom, the NNP atoms staged in LDS:
//                 F_j and a per-block energy partial;
//   NNP side      one thread per NNP atom for one chunk of MM atoms staged
//                 in LDS: per-chunk partial F_i;
//                 (both sides run as the two halves of one launch)
//   k_couple_sum  fixed-shape sums of the partials into F_i and E.
//
// Each pair is therefore evaluated twice (once per side), which costs
// ~30 flops per pair and saves every cross-thread reduction of the scatter.
#include <hip/hip_runtime.h>

#include "nnp_internal.h"

namespace nnp {

// per-atom operands staged in LDS: x, y, z, q, sigma/2, sqrt(eps)
constexpr int kCoupleVals = 6;
constexpr int kMmBlock = 256;

template <typename T> __device__ inline T c_rsqrt(T x);
template <> __device__ inline float c_rsqrt<float>(float x) { return __builtin_amdgcn_rsqf(x); }
template <> __device__ inline double c_rsqrt<double>(double x) { return 1.0 / sqrt(x); }

// energy of the pair and (dV/dr)/r
template <typename T>
__device__ inline void couple_pair(T k, T r2, T qq, T sig, T se, T& v, T& dvr) {
    const T ri = c_rsqrt(r2);
    const T ri2 = ri * ri;
    const T coul = k * qq * ri;
    const T s2 = sig * sig * ri2;
    const T s6 = s2 * s2 * s2, s12 = s6 * s6;
    const T e4 = T(4) * se;   // 4 eps_ij
    v = coul + e4 * (s12 - s6);
    dvr = (-coul - e4 * (T(12) * s12 - T(6) * s6)) * ri2;
}

template <typename T>
__device__ inline void load_atom(const T* __restrict__ x, const T* __restrict__ par, int i, T out[kCoupleVals]) {
    out[0] = x[3 * (size_t)i];
    out[1] = x[3 * (size_t)i + 1];
    out[2] = x[3 * (size_t)i + 2];
    out[3] = par[3 * (size_t)i];
    out[4] = T(0.5) * par[3 * (size_t)i + 1];
    out[5] = sqrt(par[3 * (size_t)i + 2]);
}

// MM side: four lanes per MM atom j, each over every fourth NNP atom (staged
// in LDS, s = [6][n_nnp]), combined by a fixed two-step shuffle tree; F_j and
// the block's energy partial.
constexpr int kMmLanes = 4;
constexpr int kMmPerBlock = kMmBlock / kMmLanes;   // MM atoms per workgroup
static_assert(kMmPerBlock == kCoupleMmPerBlock, "energy partials sized by the handle");

template <typename T>
__device__ inline void couple_mm_side(int blk, int n_nnp, const T* __restrict__ x_nnp,
                                      const T* __restrict__ par_nnp, int n_mm, const T* __restrict__ x_mm,
                                      const T* __restrict__ par_mm, T k, T rc2, T* __restrict__ F_mm,
                                      int accumulate, double* __restrict__ e_part, T* s, double* red) {
    for (int i = threadIdx.x; i < n_nnp; i += blockDim.x) {
        T a[kCoupleVals];
        load_atom(x_nnp, par_nnp, i, a);
#pragma unroll
        for (int v = 0; v < kCoupleVals; ++v) s[v * n_nnp + i] = a[v];
    }
    __syncthreads();
    const int j = blk * kMmPerBlock + (int)(threadIdx.x / kMmLanes), sub = threadIdx.x % kMmLanes;
    const bool act = j < n_mm;
    T f0 = 0, f1 = 0, f2 = 0;
    double e = 0.0;
    if (act) {
        T b[kCoupleVals];
        load_atom(x_mm, par_mm, j, b);
        for (int i = sub; i < n_nnp; i += kMmLanes) {
            const T d0 = b[0] - s[i], d1 = b[1] - s[n_nnp + i], d2 = b[2] - s[2 * n_nnp + i];
            const T r2 = d0 * d0 + d1 * d1 + d2 * d2;
            if (rc2 > T(0) && r2 >= rc2) continue;
            T v, dvr;
            couple_pair(k, r2, s[3 * n_nnp + i] * b[3], s[4 * n_nnp + i] + b[4], s[5 * n_nnp + i] * b[5], v,
                        dvr);
            e += (double)v;
            f0 -= dvr * d0;
            f1 -= dvr * d1;
            f2 -= dvr * d2;
        }
    }
    // the four lanes of one MM atom are adjacent
#pragma unroll
    for (int o = 1; o < kMmLanes; o <<= 1) {
        f0 += __shfl_xor(f0, o);
        f1 += __shfl_xor(f1, o);
        f2 += __shfl_xor(f2, o);
        e += __shfl_xor(e, o);
    }
    if (act && sub == 0) {
        T* F = F_mm + 3 * (size_t)j;
        F[0] = (accumulate ? F[0] : T(0)) + f0;
        F[1] = (accumulate ? F[1] : T(0)) + f1;
        F[2] = (accumulate ? F[2] : T(0)) + f2;
    }
    if (sub != 0) e = 0.0;
    for (int o = 32; o > 0; o >>= 1) e += __shfl_xor(e, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = e;
    __syncthreads();
    if (threadIdx.x == 0) e_part[blk] = (red[0] + red[1]) + (red[2] + red[3]);
}

// NNP side: each wave takes one chunk of MM atoms (staged in its own LDS
// slice) and one group of 64 NNP atoms, a thread per NNP atom; partial F_i of
// the chunk, stored component-major ([3 n_nnp][n_chunks]).
template <typename T>
__device__ inline void couple_nnp_side(int blk, int n_cg, int n_chunks, int n_nnp, const T* __restrict__ x_nnp,
                                       const T* __restrict__ par_nnp, int n_mm, const T* __restrict__ x_mm,
                                       const T* __restrict__ par_mm, T k, T rc2, int chunk,
                                       T* __restrict__ f_part, T* s_all) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = blk / n_cg, c = (blk % n_cg) * 4 + wave;
    if (c >= n_chunks) return;
    T* s = s_all + (size_t)wave * kCoupleVals * chunk;
    const int j0 = c * chunk, nj = min(chunk, n_mm - j0);
    for (int t = lane; t < nj; t += 64) {
        T b[kCoupleVals];
        load_atom(x_mm, par_mm, j0 + t, b);
#pragma unroll
        for (int v = 0; v < kCoupleVals; ++v) s[v * chunk + t] = b[v];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int i = g * 64 + lane;
    if (i >= n_nnp) return;
    T a[kCoupleVals];
    load_atom(x_nnp, par_nnp, i, a);
    T f[2][3] = {{0, 0, 0}, {0, 0, 0}};
    int t = 0;
    for (; t < nj; ++t) {
        const int u = t & 1;
        const T d0 = s[t] - a[0], d1 = s[chunk + t] - a[1], d2 = s[2 * chunk + t] - a[2];
        const T r2 = d0 * d0 + d1 * d1 + d2 * d2;
        if (rc2 > T(0) && r2 >= rc2) continue;
        T v, dvr;
        couple_pair(k, r2, a[3] * s[3 * chunk + t], a[4] + s[4 * chunk + t], a[5] * s[5 * chunk + t], v, dvr);
        // F_i = -dV/dx_i = +(dV/dr)(d/r)
        f[u][0] += dvr * d0;
        f[u][1] += dvr * d1;
        f[u][2] += dvr * d2;
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) f_part[(size_t)(3 * i + q) * n_chunks + c] = f[0][q] + f[1][q];
}

// both sides in one launch: blocks [0, n_eblk) take the MM side, the rest
// the NNP side (n_groups x n_cg blocks of four chunks)
template <typename T>
__global__ __launch_bounds__(kMmBlock) void k_couple_pairs(int n_eblk, int n_cg, int n_chunks, int n_nnp,
                                                           const T* __restrict__ x_nnp,
                                                           const T* __restrict__ par_nnp, int n_mm,
                                                           const T* __restrict__ x_mm,
                                                           const T* __restrict__ par_mm, T k, T rc2,
                                                           int chunk, T* __restrict__ F_mm, int accumulate,
                                                           double* __restrict__ e_part,
                                                           T* __restrict__ f_part) {
    extern __shared__ __align__(16) char smem[];
    __shared__ double red[kMmBlock / 64];
    if ((int)blockIdx.x < n_eblk)
        couple_mm_side(blockIdx.x, n_nnp, x_nnp, par_nnp, n_mm, x_mm, par_mm, k, rc2, F_mm, accumulate,
                       e_part, (T*)smem, red);
    else
        couple_nnp_side(blockIdx.x - n_eblk, n_cg, n_chunks, n_nnp, x_nnp, par_nnp, n_mm, x_mm, par_mm, k,
                        rc2, chunk, f_part, (T*)smem);
}

// One workgroup per NNP force component (and one for the energy): the
// threads stride over the partials, then a fixed-shape tree combines them,
// so the sum is the same on every run.
template <typename T>
__global__ __launch_bounds__(256) void k_couple_sum(int n_nnp, int n_chunks, const T* __restrict__ f_part,
                                                    int n_eblk, const double* __restrict__ e_part,
                                                    T* __restrict__ F_nnp, double* __restrict__ E,
                                                    int accumulate) {
    __shared__ double red[4];
    const int t = blockIdx.x;                 // component (t < 3 n_nnp) or the energy
    const bool energy = t == 3 * n_nnp;
    const int n = energy ? n_eblk : n_chunks;
    double v = 0.0;
    for (int c = threadIdx.x; c < n; c += blockDim.x)
        v += energy ? e_part[c] : (double)f_part[(size_t)t * n_chunks + c];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        v = (red[0] + red[1]) + (red[2] + red[3]);
        if (energy) *E = accumulate ? *E + v : v;
        else F_nnp[t] = accumulate ? F_nnp[t] + (T)v : (T)v;
    }
}

template <typename T>
hipError_t launch_coupling(const CouplingShape& cs, int n_nnp, const T* x_nnp, const T* par_nnp,
                           int n_mm, const T* x_mm, const T* par_mm, double* E, T* F_nnp, T* F_mm,
                           double* e_part, T* f_part, bool accumulate, hipStream_t st) {
    const T k = (T)cs.coulomb_k, rc2 = (T)(cs.cutoff > 0 ? cs.cutoff * cs.cutoff : 0.0);
    const int n_eblk = n_mm > 0 ? (n_mm + kMmPerBlock - 1) / kMmPerBlock : 0;
    const int n_chunks = n_mm > 0 ? (n_mm + cs.chunk - 1) / cs.chunk : 0;
    if (n_eblk > 0) {
        const int n_groups = n_nnp > 0 ? (n_nnp + 63) / 64 : 0, n_cg = (n_chunks + 3) / 4;
        const size_t lds = sizeof(T) * kCoupleVals * std::max((size_t)std::max(n_nnp, 1), (size_t)4 * cs.chunk);
        hipError_t e = ensure_lds((const void*)k_couple_pairs<T>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_couple_pairs<T>, dim3(n_eblk + n_groups * n_cg), dim3(kMmBlock), lds, st,
                           n_eblk, n_cg, n_chunks, n_nnp, x_nnp, par_nnp, n_mm, x_mm, par_mm, k, rc2,
                           cs.chunk, F_mm, accumulate ? 1 : 0, e_part, f_part);
    }
    hipLaunchKernelGGL(k_couple_sum<T>, dim3(3 * n_nnp + 1), dim3(256), 0, st, n_nnp,
                       n_nnp > 0 ? n_chunks : 0, f_part, n_eblk, e_part, F_nnp, E, accumulate ? 1 : 0);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free coupling entry point: the per-block energy
// partials and the per-chunk NNP force partials live in this array instead
// of a handle's workspace.  Every GPU the library runs on holds its own copy
// for the lifetime of the process; host code uses only the device address
// obtained below, never the array's name.
static __device__ __align__(256) unsigned char scratch[kCoupleScratchBytes];

hipError_t coupling_scratch(void** ptr) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        // raise the pair kernel's dynamic-LDS limit now (its largest size),
        // so later calls do no host-side set-up
        e = ensure_lds((const void*)k_couple_pairs<float>, sizeof(float) * kCoupleVals * 4 * 512);
        if (e == hipSuccess)
            e = ensure_lds((const void*)k_couple_pairs<double>, sizeof(double) * kCoupleVals * 4 * 512);
        if (e != hipSuccess) return e;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

template hipError_t launch_coupling<float>(const CouplingShape&, int, const float*, const float*, int,
                                           const float*, const float*, double*, float*, float*,
                                           double*, float*, bool, hipStream_t);
template hipError_t launch_coupling<double>(const CouplingShape&, int, const double*, const double*,
                                            int, const double*, const double*, double*, double*,
                                            double*, double*, double*, bool, hipStream_t);

}  // namespace nnp
