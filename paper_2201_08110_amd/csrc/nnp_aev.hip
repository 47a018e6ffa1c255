// nnp_aev.hip -- featuriser side of the path on gfx950: element bucketing,
// neighbour lists, AEV forward, AEV backward + force scatter, energy sums.
//
// The featuriser is the ANI form of the modified Behler-Parrinello symmetry
// functions the paper names (Introduction; Methods, software stack), with a
// cosine cutoff; forces are F = -dV/dx (Methods, Eq. 3) by the exact chain
// rule through the same terms.  Work mapping (wave64):
//   * a workgroup owns one molecule chunk; the molecule's coordinates and
//     element labels are staged in LDS;
//   * one wavefront per central atom; radial work is spread over
//     (neighbour, 4-shift group) lanes, angular work over neighbour pairs
//     {j<k}, enumerated in-wave from the atom's angular neighbour list (no
//     triple list is materialised);
//   * the 1008-wide AEV row (forward) or dE/dAEV row (backward) of the atom
//     lives in the wave's LDS slice; the backward accumulates the molecule's
//     forces in LDS and adds them to global memory once per workgroup.
#include "nnp_internal.h"

namespace nnp {

// --------------------------------------------------------------------------
// math in the featuriser's type
__device__ inline float m_exp(float x) { return expf(x); }
__device__ inline double m_exp(double x) { return exp(x); }
__device__ inline float m_cos(float x) { return cosf(x); }
__device__ inline double m_cos(double x) { return cos(x); }
__device__ inline float m_sin(float x) { return sinf(x); }
__device__ inline double m_sin(double x) { return sin(x); }
__device__ inline float m_sqrt(float x) { return sqrtf(x); }
__device__ inline double m_sqrt(double x) { return sqrt(x); }
// x^p for x in [0, 1], p > 0 (0^p = 0)
__device__ inline float m_powu(float x, float p) { return x > 0.f ? exp2f(p * log2f(x)) : 0.f; }
__device__ inline double m_powu(double x, double p) { return x > 0.0 ? pow(x, p) : 0.0; }

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline void lds_add(float* p, float v) { atomicAdd(p, v); }
__device__ inline void lds_add(double* p, double v) { atomicAdd(p, v); }
__device__ inline void gbl_add(float* p, float v) { unsafeAtomicAdd(p, v); }
__device__ inline void gbl_add(double* p, double v) { unsafeAtomicAdd(p, v); }

__device__ inline int lane_id() { return __lane_id(); }

// upper-triangle index of the unordered element pair (b, c)
__device__ inline int pair_index(int b, int c, int S) {
    int lo = b < c ? b : c, hi = b < c ? c : b;
    return lo * S - (lo * (lo - 1)) / 2 + (hi - lo);
}

// pair number p of the n(n-1)/2 pairs {j<k} of 0..n-1, row-major in j
__host__ __device__ inline void decode_pair(int p, int n, int& j, int& k) {
    float t = (float)(2 * n - 1);
    int jj = (int)((t - sqrtf(fmaxf(t * t - 8.0f * (float)p, 0.0f))) * 0.5f);
    jj = jj < 0 ? 0 : (jj > n - 2 ? n - 2 : jj);
    // start(j) = j (2n - j - 1) / 2
    while (jj > 0 && (jj * (2 * n - jj - 1)) / 2 > p) --jj;
    while (jj + 1 <= n - 2 && ((jj + 1) * (2 * n - jj - 2)) / 2 <= p) ++jj;
    j = jj;
    k = p - (jj * (2 * n - jj - 1)) / 2 + jj + 1;
}

// ==========================================================================
// prep: one workgroup of 1024 threads.  Molecule sanity checks, atom ->
// molecule map, element histogram, padded bucket starts, a stable counting
// sort of atoms into element buckets (row_of_atom / atom_of_row) and the
// element of every row tile.
__global__ __launch_bounds__(1024) void k_prep(int A, int B, int S, int row_tile, int max_apm,
                                               int Rcap, const int32_t* __restrict__ mol_off,
                                               const int32_t* __restrict__ species,
                                               int32_t* __restrict__ row_of_atom,
                                               int32_t* __restrict__ atom_of_row,
                                               int32_t* __restrict__ mol_of_atom,
                                               int32_t* __restrict__ tile_species,
                                               BucketInfo* __restrict__ info,
                                               int32_t* __restrict__ flag) {
    __shared__ int cnt[kMaxSpecies];
    __shared__ int base[kMaxSpecies + 1];
    __shared__ int running[kMaxSpecies];
    __shared__ int wcnt[16][kMaxSpecies];
    const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
    if (tid < kMaxSpecies) cnt[tid] = 0;
    if (tid == 0 && (mol_off[0] != 0 || mol_off[B] != A)) atomicOr(flag, FLAG_CAPACITY);
    __syncthreads();
    for (int b = tid; b < B; b += blockDim.x) {
        int a0 = mol_off[b], a1 = mol_off[b + 1];
        if (a0 < 0 || a1 < a0 || a1 > A || a1 - a0 > max_apm) {
            atomicOr(flag, FLAG_CAPACITY);
            continue;
        }
        for (int a = a0; a < a1; ++a) mol_of_atom[a] = b;
    }
    for (int a = tid; a < A; a += blockDim.x) {
        int s = species[a];
        if (s < 0 || s >= S) {
            atomicOr(flag, FLAG_SPECIES);
            s = 0;
        }
        atomicAdd(&cnt[s], 1);
    }
    __syncthreads();
    if (tid == 0) {
        base[0] = 0;
        for (int s = 0; s < S; ++s) {
            base[s + 1] = base[s] + ((cnt[s] + row_tile - 1) / row_tile) * row_tile;
            info->count[s] = cnt[s];
            running[s] = 0;
        }
        for (int s = 0; s <= S; ++s) info->off[s] = base[s];
        int rows = base[S];
        if (rows > Rcap) {
            atomicOr(flag, FLAG_CAPACITY);
            rows = 0;
        }
        info->rows = rows;
    }
    __syncthreads();
    const int rows = base[S] <= Rcap ? base[S] : 0;
    for (int t = tid; t < Rcap / row_tile; t += blockDim.x) {
        int r = t * row_tile, s = -1;
        if (r < rows)
            for (int q = 0; q < S; ++q)
                if (base[q] <= r && r < base[q + 1]) s = q;
        tile_species[t] = s;
    }
    for (int r = tid; r < rows; r += blockDim.x) atom_of_row[r] = -1;
    __syncthreads();
    if (rows == 0 && A > 0) return;
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int c0 = 0; c0 < A; c0 += blockDim.x) {
        int a = c0 + tid;
        int s = -1;
        if (a < A) {
            s = species[a];
            if (s < 0 || s >= S) s = 0;
        }
        int mypre = 0;
        for (int q = 0; q < S; ++q) {
            unsigned long long m = __ballot(s == q);
            if (lane == 0) wcnt[wave][q] = __popcll(m);
            if (s == q) mypre = __popcll(m & lt);
        }
        __syncthreads();
        if (s >= 0) {
            int pre = 0;
            for (int w = 0; w < wave; ++w) pre += wcnt[w][s];
            int row = base[s] + running[s] + pre + mypre;
            row_of_atom[a] = row;
            atom_of_row[row] = a;
        }
        __syncthreads();
        if (tid < S) {
            int add = 0;
            for (int w = 0; w < (int)(blockDim.x >> 6); ++w) add += wcnt[w][tid];
            running[tid] += add;
        }
        __syncthreads();
    }
}

template <typename P>
hipError_t launch_prep(const Shape& sh, const int32_t* mol_off, const int32_t* species,
                       Work<P>& w, hipStream_t st, const Timer& tm) {
    tm.b("prep", st);
    hipLaunchKernelGGL(k_prep, dim3(1), dim3(1024), 0, st, sh.A, sh.B, sh.S, sh.row_tile,
                       sh.max_apm, sh.Rcap, mol_off, species, w.row_of_atom, w.atom_of_row,
                       w.mol_of_atom, w.tile_species, w.info, w.flag);
    tm.e("prep", st);
    return hipGetLastError();
}

// ==========================================================================
// neighbour lists: for every atom, the local indices of the atoms of its
// molecule within rcr, those within rca first.  All pairs of the molecule are
// tested from LDS (molecules are at most kMaxAtomsPerMol atoms).  Also zeroes
// the force output.
constexpr int kChunk = 64;     // central atoms per workgroup
constexpr int kWaves = 4;

template <typename T>
__global__ __launch_bounds__(256) void k_neighbours(int A, int max_apm, int cap, T rca2, T rcr2,
                                                    const int32_t* __restrict__ mol_off,
                                                    const T* __restrict__ x, T* __restrict__ F,
                                                    uint16_t* __restrict__ nbr,
                                                    int32_t* __restrict__ nbr_cnt,
                                                    int32_t* __restrict__ flag) {
    __shared__ T sx[kMaxAtomsPerMol * 3];
    const int b = blockIdx.x;
    const int a0 = mol_off[b], n = mol_off[b + 1] - a0;
    if (n <= 0 || n > max_apm || a0 < 0 || a0 + n > A) return;
    const int i0 = blockIdx.y * kChunk;
    if (i0 >= n) return;
    const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
    for (int t = tid; t < 3 * n; t += blockDim.x) sx[t] = x[3 * (size_t)a0 + t];
    __syncthreads();
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int i1 = min(i0 + kChunk, n);
    for (int il = i0 + wave; il < i1; il += kWaves) {
        const size_t ai = (size_t)a0 + il;
        if (F && lane < 3) F[3 * ai + lane] = T(0);
        const T xi0 = sx[3 * il], xi1 = sx[3 * il + 1], xi2 = sx[3 * il + 2];
        uint16_t* out = nbr + ai * cap;
        int cntv = 0, nang = 0;
        for (int pass = 0; pass < 2; ++pass) {
            for (int j0 = 0; j0 < n; j0 += 64) {
                int j = j0 + lane;
                bool keep = false;
                if (j < n && j != il) {
                    T d0 = sx[3 * j] - xi0, d1 = sx[3 * j + 1] - xi1, d2 = sx[3 * j + 2] - xi2;
                    T r2 = d0 * d0 + d1 * d1 + d2 * d2;
                    keep = pass == 0 ? (r2 < rca2) : (r2 >= rca2 && r2 < rcr2);
                }
                unsigned long long m = __ballot(keep);
                int pos = cntv + __popcll(m & lt);
                if (keep && pos < cap) out[pos] = (uint16_t)j;
                cntv += __popcll(m);
            }
            if (pass == 0) nang = cntv;
        }
        if (lane == 0) {
            int nall = cntv;
            if (nall > cap) {
                atomicOr(flag, FLAG_CAPACITY);
                nall = cap;
                nang = nang > cap ? cap : nang;
            }
            nbr_cnt[ai] = nang | (nall << 16);
        }
    }
}

template <typename P>
hipError_t launch_neighbours(const Shape& sh, const AevConst<typename P::T>& c,
                             const int32_t* mol_off, const typename P::T* x, typename P::T* F,
                             Work<P>& w, hipStream_t st, const Timer& tm) {
    typedef typename P::T T;
    dim3 grid(sh.B, (sh.max_apm + kChunk - 1) / kChunk);
    tm.b("neighbours", st);
    hipLaunchKernelGGL(k_neighbours<T>, grid, dim3(256), 0, st, sh.A, sh.max_apm, sh.cap_nbr, c.rca2,
                       c.rcr2, mol_off, x, F, w.nbr, w.nbr_cnt, w.flag);
    tm.e("neighbours", st);
    return hipGetLastError();
}

// ==========================================================================
// shared-memory layout of the AEV kernels (dynamic LDS):
//   sx    [max_apm*3] T   molecule coordinates
//   ssp   [max_apm]  int  molecule element labels
//   sF    [max_apm*3] T   force accumulators (backward only)
//   per wave: row [Dp] T, nb [cap*4] T (dx, dy, dz, r), nsp [cap] int
//             (element), nid [cap] int (local index)
template <typename T> struct AevSmem {
    T* sx;
    int* ssp;
    T* sF;
    T* row;
    T* nb;
    int* nsp;
    int* nid;
    __device__ AevSmem(char* base, int max_apm, int Dp, int cap, int wave, bool forces) {
        size_t o = 0;
        sx = (T*)(base + o);   o += sizeof(T) * 3 * max_apm;
        sF = (T*)(base + o);   o += forces ? sizeof(T) * 3 * max_apm : 0;
        o = (o + 15) & ~size_t(15);
        row = (T*)(base + o) + (size_t)wave * Dp;   o += sizeof(T) * (size_t)kWaves * Dp;
        nb = (T*)(base + o) + (size_t)wave * cap * 4; o += sizeof(T) * (size_t)kWaves * cap * 4;
        ssp = (int*)(base + o);  o += sizeof(int) * max_apm;
        nsp = (int*)(base + o) + (size_t)wave * cap;  o += sizeof(int) * (size_t)kWaves * cap;
        nid = (int*)(base + o) + (size_t)wave * cap;
    }
    static size_t bytes(int max_apm, int Dp, int cap, bool forces) {
        size_t o = sizeof(T) * 3 * max_apm + (forces ? sizeof(T) * 3 * max_apm : 0);
        o = (o + 15) & ~size_t(15);
        o += sizeof(T) * (size_t)kWaves * Dp + sizeof(T) * (size_t)kWaves * cap * 4;
        o += sizeof(int) * max_apm + 2 * sizeof(int) * (size_t)kWaves * cap;
        return o;
    }
};

// neighbour geometry of atom il into the wave's cache; returns n_ang, n_all
template <typename T>
__device__ inline void load_neighbours(const AevSmem<T>& sm, const uint16_t* __restrict__ nb_list,
                                       int cnt, int il, int& nang, int& nall) {
    nang = cnt & 0xffff;
    nall = cnt >> 16;
    const T xi0 = sm.sx[3 * il], xi1 = sm.sx[3 * il + 1], xi2 = sm.sx[3 * il + 2];
    for (int t = lane_id(); t < nall; t += 64) {
        int j = nb_list[t];
        T d0 = sm.sx[3 * j] - xi0, d1 = sm.sx[3 * j + 1] - xi1, d2 = sm.sx[3 * j + 2] - xi2;
        sm.nb[4 * t + 0] = d0;
        sm.nb[4 * t + 1] = d1;
        sm.nb[4 * t + 2] = d2;
        sm.nb[4 * t + 3] = m_sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        sm.nsp[t] = sm.ssp[j];
        sm.nid[t] = j;
    }
}

// --------------------------------------------------------------------------
// AEV forward.  Output row of atom a goes to G[row_of_atom[a]] in the GEMM
// operand type; optionally also to aev_out[a] (atom order, unpadded).
template <typename P, int NZ>
__global__ __launch_bounds__(256) void k_aev(AevConst<typename P::T> c, int A, int max_apm, int cap,
                                             const int32_t* __restrict__ mol_off,
                                             const int32_t* __restrict__ species,
                                             const typename P::T* __restrict__ x,
                                             const uint16_t* __restrict__ nbr,
                                             const int32_t* __restrict__ nbr_cnt,
                                             const int32_t* __restrict__ row_of_atom,
                                             typename P::TS* __restrict__ G,
                                             typename P::T* __restrict__ aev_out) {
    typedef typename P::T T;
    typedef typename P::TS TS;
    extern __shared__ __align__(16) char smem[];
    const int b = blockIdx.x;
    const int a0 = mol_off[b], n = mol_off[b + 1] - a0;
    if (n <= 0 || n > max_apm || a0 < 0 || a0 + n > A) return;
    const int i0 = blockIdx.y * kChunk;
    if (i0 >= n) return;
    const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
    AevSmem<T> sm(smem, max_apm, c.Dp, cap, wave, false);
    for (int t = tid; t < 3 * n; t += blockDim.x) sm.sx[t] = x[3 * (size_t)a0 + t];
    for (int t = tid; t < n; t += blockDim.x) {
        int s = species[a0 + t];
        sm.ssp[t] = (s < 0 || s >= c.S) ? 0 : s;
    }
    __syncthreads();
    const int radial_len = c.S * kNR;
    const int i1 = min(i0 + kChunk, n);
    for (int il = i0 + wave; il < i1; il += kWaves) {
        const size_t ai = (size_t)a0 + il;
        int nang, nall;
        load_neighbours(sm, nbr + ai * cap, nbr_cnt[ai], il, nang, nall);
        for (int e = lane; e < c.Dp; e += 64) sm.row[e] = T(0);
        wave_sync();
        // radial: lane per (neighbour, group of 4 shifts)
        for (int it = lane; it < 4 * nall; it += 64) {
            const int t = it >> 2, q = it & 3;
            const T r = sm.nb[4 * t + 3];
            const T fc = T(0.5) * m_cos(c.pi_rcr * r) + T(0.5);
            T* dst = sm.row + kNR * sm.nsp[t] + 4 * q;
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const T d = r - c.shf_r[4 * q + kk];
                lds_add(dst + kk, c.radial_pref * m_exp(-c.eta_r * d * d) * fc);
            }
        }
        // angular: lane per unordered neighbour pair {j<k} of the angular list
        const int npair = nang * (nang - 1) / 2;
        for (int p = lane; p < npair; p += 64) {
            int j, k;
            decode_pair(p, nang, j, k);
            const T dj0 = sm.nb[4 * j], dj1 = sm.nb[4 * j + 1], dj2 = sm.nb[4 * j + 2];
            const T rj = sm.nb[4 * j + 3];
            const T dk0 = sm.nb[4 * k], dk1 = sm.nb[4 * k + 1], dk2 = sm.nb[4 * k + 2];
            const T rk = sm.nb[4 * k + 3];
            T cs = (dj0 * dk0 + dj1 * dk1 + dj2 * dk2) / (rj * rk);
            cs = cs > T(1) ? T(1) : (cs < T(-1) ? T(-1) : cs);
            const T cp = c.angle_scale * cs;
            const T sn = m_sqrt(T(1) - cp * cp);
            const T fcc = (T(0.5) * m_cos(c.pi_rca * rj) + T(0.5)) *
                          (T(0.5) * m_cos(c.pi_rca * rk) + T(0.5));
            const T rm = T(0.5) * (rj + rk);
            constexpr int NA = kNAZ / NZ;
            T fz[NZ];
            T fa[NA];
#pragma unroll
            for (int z = 0; z < NZ; ++z) {
                const T cz = cp * c.cos_z[z] + sn * c.sin_z[z];
                fz[z] = T(2) * m_powu(T(0.5) * (T(1) + cz), c.zeta);
            }
#pragma unroll
            for (int a = 0; a < NA; ++a) {
                const T d = rm - c.shf_a[a];
                fa[a] = m_exp(-c.eta_a * d * d) * fcc;
            }
            T* dst = sm.row + radial_len + kNAZ * pair_index(sm.nsp[j], sm.nsp[k], c.S);
#pragma unroll
            for (int a = 0; a < NA; ++a)
#pragma unroll
                for (int z = 0; z < NZ; ++z) lds_add(dst + NZ * a + z, fz[z] * fa[a]);
        }
        wave_sync();
        const size_t row = (size_t)row_of_atom[ai];
        for (int e = lane; e < c.Dp; e += 64) G[row * c.Dp + e] = Store<TS>::st(sm.row[e]);
        if (aev_out)
            for (int e = lane; e < c.D; e += 64) aev_out[ai * c.D + e] = sm.row[e];
        wave_sync();
    }
}

template <typename P>
hipError_t launch_aev(const Shape& sh, const AevConst<typename P::T>& c, const int32_t* mol_off,
                      const int32_t* species, const typename P::T* x, Work<P>& w,
                      typename P::T* aev_out, hipStream_t st, const Timer& tm) {
    typedef typename P::T T;
    dim3 grid(sh.B, (sh.max_apm + kChunk - 1) / kChunk);
    size_t lds = AevSmem<T>::bytes(sh.max_apm, c.Dp, sh.cap_nbr, false);
    auto kern = c.nZ == 4 ? k_aev<P, 4> : k_aev<P, 8>;
    hipError_t e = hipFuncSetAttribute((const void*)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    tm.b("aev", st);
    hipLaunchKernelGGL(kern, grid, dim3(256), lds, st, c, sh.A, sh.max_apm, sh.cap_nbr, mol_off,
                       species, x, w.nbr, w.nbr_cnt, w.row_of_atom, w.G, aev_out);
    tm.e("aev", st);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// AEV backward: dE/dx contracted from dE/dAEV rows (dG, already scaled to
// energy units), forces F = -dE/dx accumulated per molecule in LDS and added
// to F (zeroed by the neighbour kernel) once per workgroup.
template <typename P, int NZ>
__global__ __launch_bounds__(256) void k_forces(AevConst<typename P::T> c, int A, int max_apm, int cap,
                                                const int32_t* __restrict__ mol_off,
                                                const int32_t* __restrict__ species,
                                                const typename P::T* __restrict__ x,
                                                const uint16_t* __restrict__ nbr,
                                                const int32_t* __restrict__ nbr_cnt,
                                                const int32_t* __restrict__ row_of_atom,
                                                const typename P::TA* __restrict__ dG,
                                                typename P::T* __restrict__ F) {
    typedef typename P::T T;
    extern __shared__ __align__(16) char smem[];
    const int b = blockIdx.x;
    const int a0 = mol_off[b], n = mol_off[b + 1] - a0;
    if (n <= 0 || n > max_apm || a0 < 0 || a0 + n > A) return;
    const int i0 = blockIdx.y * kChunk;
    if (i0 >= n) return;
    const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
    AevSmem<T> sm(smem, max_apm, c.Dp, cap, wave, true);
    for (int t = tid; t < 3 * n; t += blockDim.x) {
        sm.sx[t] = x[3 * (size_t)a0 + t];
        sm.sF[t] = T(0);
    }
    for (int t = tid; t < n; t += blockDim.x) {
        int s = species[a0 + t];
        sm.ssp[t] = (s < 0 || s >= c.S) ? 0 : s;
    }
    __syncthreads();
    const int radial_len = c.S * kNR;
    const T dfc_r = -T(0.5) * c.pi_rcr, dfc_a = -T(0.5) * c.pi_rca;
    const int i1 = min(i0 + kChunk, n);
    for (int il = i0 + wave; il < i1; il += kWaves) {
        const size_t ai = (size_t)a0 + il;
        int nang, nall;
        load_neighbours(sm, nbr + ai * cap, nbr_cnt[ai], il, nang, nall);
        const size_t row = (size_t)row_of_atom[ai];
        for (int e = lane; e < c.D; e += 64) sm.row[e] = (T)dG[row * c.Dp + e];
        wave_sync();
        T fi0 = 0, fi1 = 0, fi2 = 0;   // force on the central atom, per lane
        // radial
        for (int it = lane; it < ((4 * nall + 63) & ~63); it += 64) {
            const bool act = it < 4 * nall;
            const int t = act ? (it >> 2) : 0, q = it & 3;
            T dEdr = 0;
            if (act) {
                const T r = sm.nb[4 * t + 3];
                const T fc = T(0.5) * m_cos(c.pi_rcr * r) + T(0.5);
                const T dfc = dfc_r * m_sin(c.pi_rcr * r);
                const T* g = sm.row + kNR * sm.nsp[t] + 4 * q;
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    const T d = r - c.shf_r[4 * q + kk];
                    const T ex = c.radial_pref * m_exp(-c.eta_r * d * d);
                    dEdr += g[kk] * ex * (T(-2) * c.eta_r * d * fc + dfc);
                }
            }
            // the four shift groups of one neighbour sit in adjacent lanes
            dEdr += __shfl_xor(dEdr, 1);
            dEdr += __shfl_xor(dEdr, 2);
            if (act && q == 0) {
                const T inv = T(1) / sm.nb[4 * t + 3];
                const T u0 = sm.nb[4 * t] * inv, u1 = sm.nb[4 * t + 1] * inv,
                        u2 = sm.nb[4 * t + 2] * inv;
                const int j = sm.nid[t];
                // dE/dx_j = dEdr u, dE/dx_i = -dEdr u;  F = -dE/dx
                lds_add(&sm.sF[3 * j + 0], -dEdr * u0);
                lds_add(&sm.sF[3 * j + 1], -dEdr * u1);
                lds_add(&sm.sF[3 * j + 2], -dEdr * u2);
                fi0 += dEdr * u0;
                fi1 += dEdr * u1;
                fi2 += dEdr * u2;
            }
        }
        // angular
        const int npair = nang * (nang - 1) / 2;
        for (int p = lane; p < npair; p += 64) {
            int j, k;
            decode_pair(p, nang, j, k);
            const T rj = sm.nb[4 * j + 3], rk = sm.nb[4 * k + 3];
            const T ij = T(1) / rj, ik = T(1) / rk;
            const T uj0 = sm.nb[4 * j] * ij, uj1 = sm.nb[4 * j + 1] * ij, uj2 = sm.nb[4 * j + 2] * ij;
            const T uk0 = sm.nb[4 * k] * ik, uk1 = sm.nb[4 * k + 1] * ik, uk2 = sm.nb[4 * k + 2] * ik;
            T cs = uj0 * uk0 + uj1 * uk1 + uj2 * uk2;
            cs = cs > T(1) ? T(1) : (cs < T(-1) ? T(-1) : cs);
            const T cp = c.angle_scale * cs;
            const T sn = m_sqrt(T(1) - cp * cp);
            const T fcj = T(0.5) * m_cos(c.pi_rca * rj) + T(0.5);
            const T fck = T(0.5) * m_cos(c.pi_rca * rk) + T(0.5);
            const T dfcj = dfc_a * m_sin(c.pi_rca * rj);
            const T dfck = dfc_a * m_sin(c.pi_rca * rk);
            const T fcc = fcj * fck;
            const T rm = T(0.5) * (rj + rk);
            const T* g = sm.row + radial_len + kNAZ * pair_index(sm.nsp[j], sm.nsp[k], c.S);
            constexpr int NA = kNAZ / NZ;
            T fz[NZ], dfz[NZ];
#pragma unroll
            for (int z = 0; z < NZ; ++z) {
                const T cz = cp * c.cos_z[z] + sn * c.sin_z[z];
                const T h = T(0.5) * (T(1) + cz);
                const T hp = m_powu(h, c.zeta - T(1));
                fz[z] = T(2) * hp * h;
                // d cos(theta'-t)/dc = s (cos t - c' sin t / sqrt(1 - c'^2))
                const T dcz = c.angle_scale * (c.cos_z[z] - cp * c.sin_z[z] / sn);
                dfz[z] = c.zeta * hp * dcz;
            }
            T Dc = 0, Drj = 0, Drk = 0;
#pragma unroll
            for (int a = 0; a < NA; ++a) {
                const T d = rm - c.shf_a[a];
                const T fa = m_exp(-c.eta_a * d * d);
                const T dfa_half = -c.eta_a * d * fa;   // d fa / d r_ij (= d/d r_ik)
                T sg = 0, sgd = 0;
#pragma unroll
                for (int z = 0; z < NZ; ++z) {
                    const T gg = g[NZ * a + z];
                    sg += gg * fz[z];
                    sgd += gg * dfz[z];
                }
                Dc += sgd * fa * fcc;
                Drj += sg * (dfa_half * fcc + fa * dfcj * fck);
                Drk += sg * (dfa_half * fcc + fa * fcj * dfck);
            }
            // dc/dx_j = (u_k - c u_j)/r_j ; dc/dx_k = (u_j - c u_k)/r_k
            const T gj0 = Drj * uj0 + Dc * (uk0 - cs * uj0) * ij;
            const T gj1 = Drj * uj1 + Dc * (uk1 - cs * uj1) * ij;
            const T gj2 = Drj * uj2 + Dc * (uk2 - cs * uj2) * ij;
            const T gk0 = Drk * uk0 + Dc * (uj0 - cs * uk0) * ik;
            const T gk1 = Drk * uk1 + Dc * (uj1 - cs * uk1) * ik;
            const T gk2 = Drk * uk2 + Dc * (uj2 - cs * uk2) * ik;
            const int jj = sm.nid[j], kk = sm.nid[k];
            lds_add(&sm.sF[3 * jj + 0], -gj0);
            lds_add(&sm.sF[3 * jj + 1], -gj1);
            lds_add(&sm.sF[3 * jj + 2], -gj2);
            lds_add(&sm.sF[3 * kk + 0], -gk0);
            lds_add(&sm.sF[3 * kk + 1], -gk1);
            lds_add(&sm.sF[3 * kk + 2], -gk2);
            fi0 += gj0 + gk0;
            fi1 += gj1 + gk1;
            fi2 += gj2 + gk2;
        }
        for (int off = 32; off > 0; off >>= 1) {
            fi0 += __shfl_xor(fi0, off);
            fi1 += __shfl_xor(fi1, off);
            fi2 += __shfl_xor(fi2, off);
        }
        if (lane == 0) {
            lds_add(&sm.sF[3 * il + 0], fi0);
            lds_add(&sm.sF[3 * il + 1], fi1);
            lds_add(&sm.sF[3 * il + 2], fi2);
        }
        wave_sync();
    }
    __syncthreads();
    for (int t = tid; t < 3 * n; t += blockDim.x) {
        T v = sm.sF[t];
        if (v != T(0)) gbl_add(&F[3 * (size_t)a0 + t], v);
    }
}

template <typename P>
hipError_t launch_forces(const Shape& sh, const AevConst<typename P::T>& c,
                         const int32_t* mol_off, const int32_t* species, const typename P::T* x,
                         Work<P>& w, typename P::T* F, hipStream_t st, const Timer& tm) {
    typedef typename P::T T;
    dim3 grid(sh.B, (sh.max_apm + kChunk - 1) / kChunk);
    size_t lds = AevSmem<T>::bytes(sh.max_apm, c.Dp, sh.cap_nbr, true);
    auto kern = c.nZ == 4 ? k_forces<P, 4> : k_forces<P, 8>;
    hipError_t e = hipFuncSetAttribute((const void*)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    tm.b("forces", st);
    hipLaunchKernelGGL(kern, grid, dim3(256), lds, st, c, sh.A, sh.max_apm, sh.cap_nbr,
                       mol_off, species, x, w.nbr, w.nbr_cnt, w.row_of_atom, w.dG, F);
    tm.e("forces", st);
    return hipGetLastError();
}

// ==========================================================================
// energies: one wave per molecule, FP64 sum of the atomic energies in a fixed
// order.  e_atom = scale * ( mean_m (sum_t Epart + b4) ) + sae_scaled.
template <typename P>
__global__ __launch_bounds__(256) void k_energy(int A, int B, int M, int NT, double scale,
                                                const int32_t* __restrict__ mol_off,
                                                const int32_t* __restrict__ species, int S,
                                                const int32_t* __restrict__ row_of_atom,
                                                const typename P::TA* __restrict__ Epart,
                                                const typename P::TA* __restrict__ b4,
                                                const typename P::TA* __restrict__ sae,
                                                double* __restrict__ E) {
    const int b = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = lane_id();
    if (b >= B) return;
    int a0 = mol_off[b], a1 = mol_off[b + 1];
    if (a0 < 0 || a1 < a0 || a1 > A) a1 = a0 = 0;
    double acc = 0.0;
    for (int a = a0 + lane; a < a1; a += 64) {
        int s = species[a];
        s = (s < 0 || s >= S) ? 0 : s;
        const size_t row = (size_t)row_of_atom[a];
        double e = 0.0;
        for (int m = 0; m < M; ++m) {
            double em = (double)b4[s * M + m];
            for (int t = 0; t < NT; ++t) em += (double)Epart[(row * M + m) * NT + t];
            e += em;
        }
        acc += scale * (e / M) + (double)sae[s];
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0) E[b] = (a1 > a0) ? acc : 0.0;
}

template <typename P>
hipError_t launch_energy(const Shape& sh, const DevWeights<P>& wt, const int32_t* mol_off,
                         const int32_t* species, Work<P>& w, double* E, hipStream_t st,
                         const Timer& tm) {
    tm.b("energy", st);
    hipLaunchKernelGGL(k_energy<P>, dim3((sh.B + 3) / 4), dim3(256), 0, st, sh.A, sh.B, sh.M,
                       sh.H3 / 64, sh.energy_scale, mol_off, species, sh.S, w.row_of_atom,
                       w.Epart, wt.b4, wt.sae, E);
    tm.e("energy", st);
    return hipGetLastError();
}

#define NNP_INST(P)                                                                            \
    template hipError_t launch_prep<P>(const Shape&, const int32_t*, const int32_t*, Work<P>&,  \
                                       hipStream_t, const Timer&);                             \
    template hipError_t launch_neighbours<P>(const Shape&, const AevConst<P::T>&,              \
                                             const int32_t*, const P::T*, P::T*, Work<P>&,     \
                                             hipStream_t, const Timer&);                       \
    template hipError_t launch_aev<P>(const Shape&, const AevConst<P::T>&, const int32_t*,     \
                                      const int32_t*, const P::T*, Work<P>&, P::T*,            \
                                      hipStream_t, const Timer&);                              \
    template hipError_t launch_forces<P>(const Shape&, const AevConst<P::T>&, const int32_t*,  \
                                         const int32_t*, const P::T*, Work<P>&, P::T*,         \
                                         hipStream_t, const Timer&);                           \
    template hipError_t launch_energy<P>(const Shape&, const DevWeights<P>&, const int32_t*,   \
                                         const int32_t*, Work<P>&, double*, hipStream_t,       \
                                         const Timer&);

NNP_INST(PrecF64)
NNP_INST(PrecF32)
NNP_INST(PrecBF16)

}  // namespace nnp
