// nnp_coupling.hip -- the NNP-MM coupling term of an NNP/MM step.
//
// Mechanical embedding (Methods, Eq. 4): every NNP atom i interacts with
// every MM atom j through a Coulomb term k q_i q_j / r and a 12-6
// Lennard-Jones term 4 eps_ij ((sigma_ij/r)^12 - (sigma_ij/r)^6), with
// Lorentz-Berthelot pair parameters sigma_ij = (sigma_i + sigma_j)/2,
// eps_ij = sqrt(eps_i eps_j) and an optional plain cutoff.  Forces act on both
// sides.  Both force sums are formed without atomics and in a fixed order:
//
//   k_couple_mm   one thread per MM atom, the NNP atoms staged in LDS:
//                 F_j and a per-block energy partial;
//   k_couple_nnp  one thread per NNP atom for one chunk of MM atoms staged
//                 in LDS: per-chunk partial F_i;
//   k_couple_sum  fixed-order sums of the partials into F_i and E.
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
    const T ri2 = T(1) / r2;
    const T ri = c_rsqrt(r2);
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

template <typename T>
__global__ __launch_bounds__(kMmBlock) void k_couple_mm(int n_nnp, const T* __restrict__ x_nnp,
                                                        const T* __restrict__ par_nnp, int n_mm,
                                                        const T* __restrict__ x_mm,
                                                        const T* __restrict__ par_mm, T k, T rc2,
                                                        T* __restrict__ F_mm, int accumulate,
                                                        double* __restrict__ e_part) {
    extern __shared__ __align__(16) char smem[];
    T* s = (T*)smem;   // [kCoupleVals][n_nnp]
    __shared__ double red[kMmBlock / 64];
    for (int i = threadIdx.x; i < n_nnp; i += blockDim.x) {
        T a[kCoupleVals];
        load_atom(x_nnp, par_nnp, i, a);
#pragma unroll
        for (int v = 0; v < kCoupleVals; ++v) s[v * n_nnp + i] = a[v];
    }
    __syncthreads();
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    double e = 0.0;
    if (j < n_mm) {
        T b[kCoupleVals];
        load_atom(x_mm, par_mm, j, b);
        T f0 = 0, f1 = 0, f2 = 0;
        for (int i = 0; i < n_nnp; ++i) {
            const T d0 = b[0] - s[i], d1 = b[1] - s[n_nnp + i], d2 = b[2] - s[2 * n_nnp + i];
            const T r2 = d0 * d0 + d1 * d1 + d2 * d2;
            if (rc2 > T(0) && r2 >= rc2) continue;
            T v, dvr;
            couple_pair(k, r2, s[3 * n_nnp + i] * b[3], s[4 * n_nnp + i] + b[4], s[5 * n_nnp + i] * b[5], v, dvr);
            e += (double)v;
            f0 -= dvr * d0;
            f1 -= dvr * d1;
            f2 -= dvr * d2;
        }
        T* F = F_mm + 3 * (size_t)j;
        if (accumulate) {
            F[0] += f0;
            F[1] += f1;
            F[2] += f2;
        } else {
            F[0] = f0;
            F[1] = f1;
            F[2] = f2;
        }
    }
    for (int o = 32; o > 0; o >>= 1) e += __shfl_xor(e, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = e;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
        e_part[blockIdx.x] = t;
    }
}

template <typename T>
__global__ __launch_bounds__(64) void k_couple_nnp(int n_nnp, const T* __restrict__ x_nnp,
                                                   const T* __restrict__ par_nnp, int n_mm,
                                                   const T* __restrict__ x_mm,
                                                   const T* __restrict__ par_mm, T k, T rc2,
                                                   int chunk, T* __restrict__ f_part) {
    extern __shared__ __align__(16) char smem[];
    T* s = (T*)smem;   // [kCoupleVals][chunk]
    const int c = blockIdx.y, j0 = c * chunk, nj = min(chunk, n_mm - j0);
    for (int t = threadIdx.x; t < nj; t += blockDim.x) {
        T b[kCoupleVals];
        load_atom(x_mm, par_mm, j0 + t, b);
#pragma unroll
        for (int v = 0; v < kCoupleVals; ++v) s[v * chunk + t] = b[v];
    }
    __syncthreads();
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_nnp) return;
    T a[kCoupleVals];
    load_atom(x_nnp, par_nnp, i, a);
    T f0 = 0, f1 = 0, f2 = 0;
    for (int t = 0; t < nj; ++t) {
        const T d0 = s[t] - a[0], d1 = s[chunk + t] - a[1], d2 = s[2 * chunk + t] - a[2];
        const T r2 = d0 * d0 + d1 * d1 + d2 * d2;
        if (rc2 > T(0) && r2 >= rc2) continue;
        T v, dvr;
        couple_pair(k, r2, a[3] * s[3 * chunk + t], a[4] + s[4 * chunk + t], a[5] * s[5 * chunk + t], v, dvr);
        // F_i = -dV/dx_i = +(dV/dr)(d/r)
        f0 += dvr * d0;
        f1 += dvr * d1;
        f2 += dvr * d2;
    }
    T* P = f_part + ((size_t)c * n_nnp + i) * 3;
    P[0] = f0;
    P[1] = f1;
    P[2] = f2;
}

template <typename T>
__global__ __launch_bounds__(256) void k_couple_sum(int n_nnp, int n_chunks, const T* __restrict__ f_part,
                                                    int n_eblk, const double* __restrict__ e_part,
                                                    T* __restrict__ F_nnp, double* __restrict__ E,
                                                    int accumulate) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < 3 * n_nnp) {
        double f = 0.0;
        for (int c = 0; c < n_chunks; ++c) f += (double)f_part[(size_t)c * n_nnp * 3 + t];
        F_nnp[t] = accumulate ? F_nnp[t] + (T)f : (T)f;
    }
    if (blockIdx.x == 0 && threadIdx.x < 64) {
        double e = 0.0;
        for (int b = threadIdx.x; b < n_eblk; b += 64) e += e_part[b];
        for (int o = 32; o > 0; o >>= 1) e += __shfl_xor(e, o);
        if (threadIdx.x == 0) *E = accumulate ? *E + e : e;
    }
}

template <typename T>
hipError_t launch_coupling(const CouplingShape& cs, int n_nnp, const T* x_nnp, const T* par_nnp,
                           int n_mm, const T* x_mm, const T* par_mm, double* E, T* F_nnp, T* F_mm,
                           double* e_part, T* f_part, bool accumulate, hipStream_t st) {
    const T k = (T)cs.coulomb_k, rc2 = (T)(cs.cutoff > 0 ? cs.cutoff * cs.cutoff : 0.0);
    const int n_eblk = n_mm > 0 ? (n_mm + kMmBlock - 1) / kMmBlock : 0;
    const int n_chunks = n_mm > 0 ? (n_mm + cs.chunk - 1) / cs.chunk : 0;
    if (n_eblk > 0) {
        hipLaunchKernelGGL(k_couple_mm<T>, dim3(n_eblk), dim3(kMmBlock),
                           sizeof(T) * kCoupleVals * (size_t)max(n_nnp, 1), st, n_nnp, x_nnp, par_nnp,
                           n_mm, x_mm, par_mm, k, rc2, F_mm, accumulate ? 1 : 0, e_part);
        if (n_nnp > 0)
            hipLaunchKernelGGL(k_couple_nnp<T>, dim3((n_nnp + 63) / 64, n_chunks), dim3(64),
                               sizeof(T) * kCoupleVals * (size_t)cs.chunk, st, n_nnp, x_nnp, par_nnp,
                               n_mm, x_mm, par_mm, k, rc2, cs.chunk, f_part);
    }
    const int nt = std::max(3 * n_nnp, 1);
    hipLaunchKernelGGL(k_couple_sum<T>, dim3((nt + 255) / 256), dim3(256), 0, st, n_nnp,
                       n_nnp > 0 ? n_chunks : 0, f_part, n_eblk, e_part, F_nnp, E, accumulate ? 1 : 0);
    return hipGetLastError();
}

template hipError_t launch_coupling<float>(const CouplingShape&, int, const float*, const float*, int,
                                           const float*, const float*, double*, float*, float*,
                                           double*, float*, bool, hipStream_t);
template hipError_t launch_coupling<double>(const CouplingShape&, int, const double*, const double*,
                                            int, const double*, const double*, double*, double*,
                                            double*, double*, double*, bool, hipStream_t);

}  // namespace nnp
