// nnp_aev.hip -- featuriser side of the path on gfx950: element bucketing,
// neighbour lists, AEV forward, AEV backward + force scatter, energy sums.
//
// The featuriser is the ANI form of the modified Behler-Parrinello symmetry
// functions the paper names (Introduction; Methods, software stack), with a
// cosine cutoff; forces are F = -dV/dx (Methods, Eq. 3) by the exact chain
// rule through the same terms.  Work mapping (wave64):
//   * a workgroup owns a chunk of one molecule's atoms; the molecule's
//     coordinates and element labels are staged in LDS;
//   * one wavefront per central atom, whose neighbour geometry (vectors,
//     distances, cutoff values) is cached in the wave's LDS slice;
//   * neighbour lists are sorted by element (angular neighbours first), so
//     radial terms of one element and angular terms of one element pair come
//     in runs: lanes accumulate a run in registers and flush it once into an
//     LDS row slice they own -- no atomics, bitwise reproducible;
//   * angular pairs {j<k} are enumerated in-wave from the angular list by a
//     triangular decode (no triple list is materialised): a lane per pair
//     computes the 8 distance and 4 angle factors, then lanes per output slot
//     expand the 32 products;
//   * the backward recomputes the terms, contracts them with the atom's
//     dE/dAEV row (LDS, element-pair blocks padded to 33 words against bank
//     conflicts), accumulates the molecule's forces in LDS and adds them to
//     global memory once per workgroup.
#include <algorithm>

#include "nnp_internal.h"

namespace nnp {

// --------------------------------------------------------------------------
// math in the featuriser's type.  FP32 uses the hardware transcendental
// instructions (v_exp_f32 = 2^x, v_log_f32 = log2, v_sin/v_cos_f32 take
// revolutions, v_sqrt_f32, v_rcp_f32; each within about 1 ulp on the ranges
// used here: arguments of cos/sin lie in [0, pi]); FP64 uses the accurate
// library functions.
__device__ inline float m_exp(float x) { return __builtin_amdgcn_exp2f(x * 1.44269504088896341f); }
__device__ inline double m_exp(double x) { return exp(x); }
__device__ inline float m_cos(float x) { return __builtin_amdgcn_cosf(x * 0.159154943091895336f); }
__device__ inline double m_cos(double x) { return cos(x); }
__device__ inline float m_sin(float x) { return __builtin_amdgcn_sinf(x * 0.159154943091895336f); }
__device__ inline double m_sin(double x) { return sin(x); }
__device__ inline float m_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ inline double m_sqrt(double x) { return sqrt(x); }
__device__ inline float m_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double m_rcp(double x) { return 1.0 / x; }
// x^p for x in [0, 1], p > 0 (0^p = 0)
__device__ inline float m_powu(float x, float p) {
    return x > 0.f ? __builtin_amdgcn_exp2f(p * __builtin_amdgcn_logf(x)) : 0.f;
}
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
__device__ inline void decode_pair(int p, int n, int& j, int& k) {
    // estimate from the hardware square root, corrected by the loops below
    float t = (float)(2 * n - 1);
    int jj = (int)((t - __builtin_amdgcn_sqrtf(fmaxf(t * t - 8.0f * (float)p, 0.0f))) * 0.5f);
    jj = jj < 0 ? 0 : (jj > n - 2 ? n - 2 : jj);
    // start(j) = j (2n - j - 1) / 2
    while (jj > 0 && (jj * (2 * n - jj - 1)) / 2 > p) --jj;
    while (jj + 1 <= n - 2 && ((jj + 1) * (2 * n - jj - 2)) / 2 <= p) ++jj;
    j = jj;
    k = p - (jj * (2 * n - jj - 1)) / 2 + jj + 1;
}

// The same pairs in rotation order: pair p = (a, a + d mod n), diagonal d
// taking n pairs each for d < n/2 (and n/2 pairs at d = n/2 when n is even).
// Consecutive p give distinct j and distinct k, so lanes that scatter into
// per-atom accumulators hit different addresses.
__device__ inline void decode_pair_rot(int p, int n, int& j, int& k) {
    const int full = n * ((n - 1) >> 1);
    int d, a;
    if (p < full) {
        d = (int)(((float)p + 0.5f) * __builtin_amdgcn_rcpf((float)n));
        a = p - d * n;
        if (a < 0) { --d; a += n; }
        if (a >= n) { ++d; a -= n; }
        d += 1;
    } else {
        d = n >> 1;
        a = p - full;
    }
    j = a;
    k = a + d >= n ? a + d - n : a + d;
}

// ==========================================================================
// Element bucketing (two kernels): per-block element counts and molecule
// checks; then, in every workgroup, the prefix of the block counts into
// padded bucket starts and a stable scatter of its atoms to their bucket rows.
// Element of atom a: the batch's label itself, or, on handles with a table
// of atomic numbers (zlut != null), the table's index of that atomic number
// (-1 when absent), written to sp_out for the later kernels.
__device__ inline int element_of(const int32_t* __restrict__ species, const int8_t* __restrict__ zlut,
                                 int32_t* __restrict__ sp_out, int a, int S) {
    int s = species[a];
    if (zlut) {
        s = (s >= 0 && s < kZLut) ? (int)zlut[s] : -1;
        sp_out[a] = s < 0 ? 0 : s;
    }
    return s < 0 || s >= S ? -1 : s;
}

// Atom range of a call: [mol_off[0], mol_off[B]).  A whole batch starts at 0
// and ends at its atom count (A, or the device count dA); a sub-batch (one
// part of a pipelined evaluation, sub = 1) may start anywhere and holds at
// most A atoms.  Per-atom arrays are indexed by absolute atom number.
__device__ inline bool atom_range(int A, int B, const int32_t* __restrict__ dA,
                                  const int32_t* __restrict__ mol_off, int sub, int& a0, int& a1) {
    a0 = mol_off[0];
    a1 = mol_off[B];
    const bool ok = sub ? (a0 >= 0 && a1 >= a0 && a1 - a0 <= A) : (a0 == 0 && a1 == (dA ? *dA : A));
    if (!ok) a1 = a0;
    return ok;
}

__global__ __launch_bounds__(1024) void k_bucket_count(int A, int B, int S, int max_apm, int sub,
                                                       const int32_t* __restrict__ dA,
                                                       const int32_t* __restrict__ mol_off,
                                                       const int32_t* __restrict__ species,
                                                       const int8_t* __restrict__ zlut,
                                                       int32_t* __restrict__ sp_out,
                                                       int32_t* __restrict__ mol_of_atom,
                                                       int32_t* __restrict__ blk_cnt,
                                                       int32_t* __restrict__ flag) {
    __shared__ int wcnt[kPrepBlock / 64][kMaxSpecies];
    const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6, blk = blockIdx.x;
    int A0, A1;
    if (!atom_range(A, B, dA, mol_off, sub, A0, A1) && blk == 0 && tid == 0) atomicOr(flag, FLAG_CAPACITY);
    // molecule ranges are checked once, by one thread per molecule
    const int b = blk * kPrepBlock + tid;
    if (b < B) {
        const int m0 = mol_off[b], m1 = mol_off[b + 1];
        if (m0 < A0 || m1 < m0 || m1 > A1 || m1 - m0 > max_apm) atomicOr(flag, FLAG_CAPACITY);
    }
    // per atom: its molecule (last b with mol_off[b] <= a, by bisection) and
    // its element, counted per wave with ballots
    const int a = A0 + blk * kPrepBlock + tid;
    int s = -1;
    if (a < A1) {
        int lo = 0, hi = B;   // mol_off[lo] <= a < mol_off[hi] for valid offsets
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (mol_off[mid] <= a) lo = mid;
            else hi = mid;
        }
        mol_of_atom[a] = lo;
        s = element_of(species, zlut, sp_out, a, S);
        if (s < 0) {
            atomicOr(flag, FLAG_SPECIES);
            s = 0;
        }
    }
    for (int q = 0; q < S; ++q) {
        const int c = __popcll(__ballot(s == q));
        if (lane == 0) wcnt[wave][q] = c;
    }
    __syncthreads();
    if (tid < S) {
        int c = 0;
        for (int w = 0; w < kPrepBlock / 64; ++w) c += wcnt[w][tid];
        blk_cnt[blk * kMaxSpecies + tid] = c;
    }
}

// Scan and scatter in one launch: every workgroup sums the count kernel's
// per-block element counts itself (totals and the prefix of the blocks
// before its own), so the padded bucket starts need no separate kernel;
// workgroup 0 also writes the bucket info, the element of every row tile and
// the padding rows.  Then the workgroup's atoms go to their rows, in atom
// order within each element (stable).
__global__ __launch_bounds__(1024) void k_bucket_place(int A, int B, int S, int sub, int nblk,
                                                       int row_tile, int Rcap,
                                                       const int32_t* __restrict__ dA,
                                                       const int32_t* __restrict__ mol_off,
                                                       const int32_t* __restrict__ species,
                                                       const int32_t* __restrict__ blk_cnt,
                                                       int32_t* __restrict__ row_of_atom,
                                                       int32_t* __restrict__ atom_of_row,
                                                       int32_t* __restrict__ tile_species,
                                                       BucketInfo* __restrict__ info,
                                                       int32_t* __restrict__ flag) {
    constexpr int NWV = kPrepBlock / 64;
    __shared__ int red[NWV][kMaxSpecies][2];
    __shared__ int tot_s[kMaxSpecies], pre_s[kMaxSpecies], base_s[kMaxSpecies + 1];
    __shared__ int wcnt[NWV][kMaxSpecies];
    const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6, blk = blockIdx.x;
    {
        // thread (chunk kc, element q): count blocks kc, kc + 128, ...
        const int q = tid & (kMaxSpecies - 1), kc = tid / kMaxSpecies;
        int tot = 0, pre = 0;
        if (q < S)
            for (int k = kc; k < nblk; k += kPrepBlock / kMaxSpecies) {
                const int v = blk_cnt[k * kMaxSpecies + q];
                tot += v;
                pre += k < blk ? v : 0;
            }
        for (int o = kMaxSpecies; o < 64; o <<= 1) {   // the lanes of one element in a wave
            tot += __shfl_xor(tot, o);
            pre += __shfl_xor(pre, o);
        }
        if (lane < kMaxSpecies) {
            red[wave][lane][0] = tot;
            red[wave][lane][1] = pre;
        }
        __syncthreads();
        if (tid < S) {
            int t = 0, p = 0;
            for (int w = 0; w < NWV; ++w) {
                t += red[w][tid][0];
                p += red[w][tid][1];
            }
            tot_s[tid] = t;
            pre_s[tid] = p;
        }
        __syncthreads();
        if (tid == 0) {
            base_s[0] = 0;
            for (int q2 = 0; q2 < S; ++q2)
                base_s[q2 + 1] = base_s[q2] + ((tot_s[q2] + row_tile - 1) / row_tile) * row_tile;
        }
        __syncthreads();
    }
    const int rows = base_s[S] <= Rcap ? base_s[S] : 0;
    if (blk == 0) {
        if (tid == 0) {
            for (int q = 0; q < S; ++q) info->count[q] = tot_s[q];
            for (int q = 0; q <= S; ++q) info->off[q] = base_s[q];
            if (base_s[S] > Rcap) atomicOr(flag, FLAG_CAPACITY);
            info->rows = rows;
        }
        for (int t = tid; t < Rcap / row_tile; t += blockDim.x) {
            const int r = t * row_tile;
            int sp = -1;
            if (r < rows)
                for (int q = 0; q < S; ++q)
                    if (base_s[q] <= r && r < base_s[q + 1]) sp = q;
            tile_species[t] = sp;
        }
        for (int q = 0; q < S; ++q)
            for (int r = base_s[q] + tot_s[q] + tid; r < base_s[q + 1] && r < rows; r += blockDim.x)
                atom_of_row[r] = -1;
    }
    int A0, A1;
    atom_range(A, B, dA, mol_off, sub, A0, A1);
    const int a = A0 + blk * kPrepBlock + tid;
    int s = -1;
    if (a < A1) {
        s = species[a];
        if (s < 0 || s >= S) s = 0;
    }
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int mypre = 0;
    for (int q = 0; q < S; ++q) {
        unsigned long long m = __ballot(s == q);
        if (lane == 0) wcnt[wave][q] = __popcll(m);
        if (s == q) mypre = __popcll(m & lt);
    }
    __syncthreads();
    if (s >= 0 && rows > 0) {
        int pre = 0;
        for (int w = 0; w < wave; ++w) pre += wcnt[w][s];
        const int row = base_s[s] + pre_s[s] + pre + mypre;
        row_of_atom[a] = row;
        atom_of_row[row] = a;
    }
}

// The three steps in one workgroup, for batches of at most kPrepBlock atoms
// and molecules (one launch instead of three on small batches); same results.
// The workgroup has one wave per 64 atoms (or molecules) of the bounds.
__global__ __launch_bounds__(1024) void k_bucket_one(int A, int B, int S, int max_apm, int row_tile,
                                                     int Rcap, int sub, const int32_t* __restrict__ dA,
                                                     const int32_t* __restrict__ mol_off,
                                                     const int32_t* __restrict__ species,
                                                     const int8_t* __restrict__ zlut,
                                                     int32_t* __restrict__ sp_out,
                                                     int32_t* __restrict__ mol_of_atom,
                                                     int32_t* __restrict__ row_of_atom,
                                                     int32_t* __restrict__ atom_of_row,
                                                     int32_t* __restrict__ tile_species,
                                                     BucketInfo* __restrict__ info,
                                                     int32_t* __restrict__ flag) {
    __shared__ int wcnt[kPrepBlock / 64][kMaxSpecies];
    __shared__ int tot[kMaxSpecies];
    __shared__ int base[kMaxSpecies + 1];
    const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
    int A0, A1;
    if (!atom_range(A, B, dA, mol_off, sub, A0, A1) && tid == 0) atomicOr(flag, FLAG_CAPACITY);
    if (tid < B) {
        const int m0 = mol_off[tid], m1 = mol_off[tid + 1];
        if (m0 < A0 || m1 < m0 || m1 > A1 || m1 - m0 > max_apm) atomicOr(flag, FLAG_CAPACITY);
    }
    const int a = A0 + tid;
    int s = -1;
    if (a < A1) {
        int lo = 0, hi = B;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (mol_off[mid] <= a) lo = mid;
            else hi = mid;
        }
        mol_of_atom[a] = lo;
        s = element_of(species, zlut, sp_out, a, S);
        if (s < 0) {
            atomicOr(flag, FLAG_SPECIES);
            s = 0;
        }
    }
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int mypre = 0;
    for (int q = 0; q < S; ++q) {
        const unsigned long long m = __ballot(s == q);
        if (lane == 0) wcnt[wave][q] = __popcll(m);
        if (s == q) mypre = __popcll(m & lt);
    }
    __syncthreads();
    // per element (lane q of wave 0): the count over the block's waves, its
    // rows padded to whole row tiles, and the offsets as a prefix scan over
    // the lanes (lane S ends with the total)
    if (wave == 0) {
        const int nwv = blockDim.x >> 6;
        int c = 0;
        if (lane < S)
            for (int w = 0; w < nwv; ++w) c += wcnt[w][lane];
        const int pc = ((c + row_tile - 1) / row_tile) * row_tile;
        int incl = pc;
        for (int d = 1; d < 2 * kMaxSpecies; d <<= 1) {
            const int v = __shfl_up(incl, d);
            if (lane >= d) incl += v;
        }
        if (lane < S) {
            tot[lane] = c;
            info->count[lane] = c;
        }
        if (lane <= S) {
            base[lane] = incl - pc;
            info->off[lane] = incl - pc;
        }
        if (lane == S) {
            int rows = incl;
            if (rows > Rcap) {
                atomicOr(flag, FLAG_CAPACITY);
                rows = 0;
            }
            info->rows = rows;
        }
    }
    __syncthreads();
    const int rows = base[S] <= Rcap ? base[S] : 0;
    for (int t = tid; t < Rcap / row_tile; t += blockDim.x) {
        const int r = t * row_tile;
        int sp = -1;
        if (r < rows)
            for (int q = 0; q < S; ++q)
                if (base[q] <= r && r < base[q + 1]) sp = q;
        tile_species[t] = sp;
    }
    for (int q = 0; q < S; ++q)
        for (int r = base[q] + tot[q] + tid; r < base[q + 1] && r < rows; r += blockDim.x) atom_of_row[r] = -1;
    if (s >= 0 && rows > 0) {
        int pre = 0;
        for (int w = 0; w < wave; ++w) pre += wcnt[w][s];
        const int row = base[s] + pre + mypre;
        row_of_atom[a] = row;
        atom_of_row[row] = a;
    }
}

// Batches whose counts live on the device: the call's launches are sized for
// the bounds B and A (host), and this kernel copies the caller's offsets of
// the counts[0] real molecules into the workspace, padding the rest of the
// bound with empty molecules at counts[1] atoms, so every later kernel sees
// a batch of B molecules of which the padding ones do nothing.  Counts
// outside the bounds set the capacity flag and run an empty batch.
__global__ __launch_bounds__(1024) void k_stage_batch(int B, int A, const int32_t* __restrict__ counts,
                                                      const int32_t* __restrict__ mol_off,
                                                      int32_t* __restrict__ moff, int32_t* __restrict__ dcnt,
                                                      int32_t* __restrict__ flag) {
    int Br = counts[0], Ar = counts[1];
    // the offsets must end at the atom count (k_bucket_count checks the rest)
    if (Br < 0 || Br > B || Ar < 0 || Ar > A || (Br > 0 ? mol_off[Br] : 0) != Ar || mol_off[0] != 0) {
        if (threadIdx.x == 0) atomicOr(flag, FLAG_CAPACITY);
        Br = 0;
        Ar = 0;
    }
    for (int b = threadIdx.x; b <= B; b += blockDim.x) moff[b] = (b <= Br && Br > 0) ? mol_off[b] : Ar;
    if (threadIdx.x == 0) {
        dcnt[0] = Br;
        dcnt[1] = Ar;
    }
}

hipError_t launch_stage_batch(int B, int A, const int32_t* counts, const int32_t* mol_off, int32_t* moff,
                              int32_t* dcnt, int32_t* flag, hipStream_t st) {
    hipLaunchKernelGGL(k_stage_batch, dim3(1), dim3(1024), 0, st, B, A, counts, mol_off, moff, dcnt, flag);
    return hipGetLastError();
}

template <typename P>
hipError_t launch_prep(const Shape& sh, const int32_t* mol_off, const int32_t* species,
                       Work<P>& w, hipStream_t st, const Timer& tm) {
    const int nblk = std::max((sh.A + kPrepBlock - 1) / kPrepBlock, (sh.B + kPrepBlock - 1) / kPrepBlock);
    int32_t* blk_cnt = w.blk;
    const int32_t* dA = sh.dev_counts ? w.dcnt + 1 : nullptr;
    tm.b("prep", st);
    if (nblk <= 1) {
        // one wave per 64 atoms (or molecules) of the bounds
        const int nt = std::min(kPrepBlock, std::max(64, (std::max(sh.A, sh.B) + 63) / 64 * 64));
        hipLaunchKernelGGL(k_bucket_one, dim3(1), dim3(nt), 0, st, sh.A, sh.B, sh.S, sh.max_apm,
                           sh.row_tile, sh.Rcap, sh.sub, dA, mol_off, species, w.zlut, w.sp, w.mol_of_atom,
                           w.row_of_atom, w.atom_of_row, w.tile_species, w.info, w.flag);
        tm.e("prep", st);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_bucket_count, dim3(nblk), dim3(kPrepBlock), 0, st, sh.A, sh.B, sh.S,
                       sh.max_apm, sh.sub, dA, mol_off, species, w.zlut, w.sp, w.mol_of_atom, blk_cnt, w.flag);
    // on handles with atomic numbers the count kernel has written the
    // element indices to w.sp
    hipLaunchKernelGGL(k_bucket_place, dim3(std::max(1, (sh.A + kPrepBlock - 1) / kPrepBlock)),
                       dim3(kPrepBlock), 0, st, sh.A, sh.B, sh.S, sh.sub, nblk, sh.row_tile, sh.Rcap, dA,
                       mol_off, w.zlut ? w.sp : species, blk_cnt, w.row_of_atom, w.atom_of_row,
                       w.tile_species, w.info, w.flag);
    tm.e("prep", st);
    return hipGetLastError();
}

// bump allocator over dynamic LDS (16-byte aligned slices)
struct LdsBump {
    char* p;
    __device__ explicit LdsBump(char* base) : p(base) {}
    template <typename X> __device__ X* take(size_t n) {
        X* r = (X*)p;
        p += (sizeof(X) * n + 15) & ~size_t(15);
        return r;
    }
};
template <typename X> inline size_t lds_bytes(size_t n) { return (sizeof(X) * n + 15) & ~size_t(15); }

// ==========================================================================
// Neighbour lists: for every atom, the local indices of the atoms of its
// molecule within rcr, those within rca first, each of the two runs sorted
// by element.  A workgroup of one wave owns up to 64 central atoms of one
// molecule, one lane per atom; the molecule's atoms are staged in LDS in
// element order (small molecules: every atom is tested) or in (element,
// cutoff cell) order (large molecules: only the <= 27 cells around the
// central atom's cell are tested), so the scan emits sorted lists, which are
// assembled in LDS and written out coalesced.  Also zeroes the forces.
constexpr int kNbrChunk = 64;  // central atoms per neighbour-list workgroup
constexpr int kChunk = 16;     // most central atoms per AEV / force workgroup (the knob picks 4..16)
constexpr int kWaves = 4;
constexpr size_t kMaxLds = 160 * 1024;   // LDS per workgroup on gfx950

constexpr int kMaxCellsPerDim = 6;  // cells per dimension (cell edge >= rcr)

template <typename T>
__device__ inline T wave_min(T v) {
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
    return v;
}
template <typename T>
__device__ inline T wave_max(T v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

template <typename T>
__global__ __launch_bounds__(64) void k_neighbours(int A, int S, int max_apm, int cell_min, int cap,
                                                   T rcr, T rca2,
                                                   T rcr2, const int32_t* __restrict__ mol_off,
                                                   const int32_t* __restrict__ species,
                                                   const T* __restrict__ x, T* __restrict__ F,
                                                   unsigned long long* __restrict__ Fq,
                                                   uint16_t* __restrict__ nbr,
                                                   int32_t* __restrict__ nbr_cnt,
                                                   int32_t* __restrict__ flag) {
    extern __shared__ __align__(16) char smem[];
    const int b = blockIdx.x;
    const int a0 = mol_off[b], n = mol_off[b + 1] - a0;
    if (n <= 0 || n > max_apm || a0 < 0 || a0 + n > A) return;
    if (n <= cell_min) return;   // listed by k_nbr_pairs
    const int i0 = blockIdx.y * kNbrChunk;
    if (i0 >= n) return;
    const int lane = lane_id();
    LdsBump lb(smem);
    T* sx = lb.take<T>(4 * (size_t)max_apm);            // staged atoms: x y z
    int* sid = lb.take<int>(max_apm);                   // local index of the k-th staged atom
    uint16_t* lst = lb.take<uint16_t>((size_t)kNbrChunk * cap);
    T* tx = lb.take<T>(3 * (size_t)max_apm);            // the molecule's x y z, input order
    int* tsp = lb.take<int>(max_apm);                   // and elements
    constexpr int kKeys = kMaxSpecies * kMaxCellsPerDim * kMaxCellsPerDim * kMaxCellsPerDim;
    int* kstart = lb.take<int>(kKeys + 1);             // bucket starts
    int* kcur = lb.take<int>(kKeys);                   // scatter cursors
    int* akey = lb.take<int>(max_apm);                 // key of every atom

    // ---- staging: atoms in (element, cell) order over a grid of cutoff
    // cells with edge >= rcr, so a central atom scans <= 27 cells
    int nc0 = 1, nc1 = 1, nc2 = 1;
    T lo0 = 0, lo1 = 0, lo2 = 0, ih0 = 0, ih1 = 0, ih2 = 0;
    // one coalesced pass over the molecule's inputs: every later pass reads LDS
    for (int t = lane; t < 3 * n; t += 64) tx[t] = x[3 * (size_t)a0 + t];
    for (int j = lane; j < n; j += 64) {
        const int s = species[a0 + j];
        tsp[j] = (s < 0 || s >= S) ? 0 : s;
    }
    wave_sync();
    {
        T mn0 = T(1e30), mn1 = T(1e30), mn2 = T(1e30), mx0 = T(-1e30), mx1 = T(-1e30), mx2 = T(-1e30);
        for (int j = lane; j < n; j += 64) {
            const T* p = tx + 3 * j;
            mn0 = fmin(mn0, p[0]); mx0 = fmax(mx0, p[0]);
            mn1 = fmin(mn1, p[1]); mx1 = fmax(mx1, p[1]);
            mn2 = fmin(mn2, p[2]); mx2 = fmax(mx2, p[2]);
        }
        lo0 = wave_min(mn0); lo1 = wave_min(mn1); lo2 = wave_min(mn2);
        const T e0 = wave_max(mx0) - lo0, e1 = wave_max(mx1) - lo1, e2 = wave_max(mx2) - lo2;
        nc0 = min(max((int)(e0 / rcr), 1), kMaxCellsPerDim);
        nc1 = min(max((int)(e1 / rcr), 1), kMaxCellsPerDim);
        nc2 = min(max((int)(e2 / rcr), 1), kMaxCellsPerDim);
        ih0 = e0 > T(0) ? T(nc0) / e0 : T(0);
        ih1 = e1 > T(0) ? T(nc1) / e1 : T(0);
        ih2 = e2 > T(0) ? T(nc2) / e2 : T(0);
        const int ncell = nc0 * nc1 * nc2, nkeys = S * ncell;
        for (int k = lane; k <= nkeys; k += 64) kstart[k] = 0;
        wave_sync();
        for (int j = lane; j < n; j += 64) {
            int s = tsp[j];
            s = (s < 0 || s >= S) ? 0 : s;
            const T* p = tx + 3 * j;
            const int c0 = min((int)((p[0] - lo0) * ih0), nc0 - 1);
            const int c1 = min((int)((p[1] - lo1) * ih1), nc1 - 1);
            const int c2 = min((int)((p[2] - lo2) * ih2), nc2 - 1);
            const int key = s * ncell + (c2 * nc1 + c1) * nc0 + c0;
            akey[j] = key;
            atomicAdd(&kstart[key + 1], 1);
        }
        wave_sync();
        // inclusive scan of the counts (lane-blocked, then across lanes)
        const int per = (nkeys + 64) / 64;
        const int k0 = lane * per, k1 = min(k0 + per, nkeys + 1);
        int run = 0;
        for (int k = k0; k < k1; ++k) run += kstart[k];
        int pre = run;
        for (int o = 1; o < 64; o <<= 1) {
            const int v = __shfl_up(pre, o);
            if (lane >= o) pre += v;
        }
        pre -= run;
        for (int k = k0; k < k1; ++k) {
            pre += kstart[k];
            kstart[k] = pre;
        }
        wave_sync();
        for (int k = lane; k < nkeys; k += 64) kcur[k] = kstart[k];
        wave_sync();
        for (int j = lane; j < n; j += 64) {
            const int pos = atomicAdd(&kcur[akey[j]], 1);
            sid[pos] = j;
            sx[4 * pos + 0] = tx[3 * j + 0];
            sx[4 * pos + 1] = tx[3 * j + 1];
            sx[4 * pos + 2] = tx[3 * j + 2];
        }
    }
    wave_sync();

    // ---- one lane per central atom: scan the staged atoms in order
    const int il = i0 + lane;
    const bool act = il < n;
    T xi0 = 0, xi1 = 0, xi2 = 0;
    if (act) {
        xi0 = x[3 * ((size_t)a0 + il) + 0];
        xi1 = x[3 * ((size_t)a0 + il) + 1];
        xi2 = x[3 * ((size_t)a0 + il) + 2];
        if (F) {
            F[3 * ((size_t)a0 + il) + 0] = T(0);
            F[3 * ((size_t)a0 + il) + 1] = T(0);
            F[3 * ((size_t)a0 + il) + 2] = T(0);
        }
        if (Fq) {
            Fq[3 * ((size_t)a0 + il) + 0] = 0ull;
            Fq[3 * ((size_t)a0 + il) + 1] = 0ull;
            Fq[3 * ((size_t)a0 + il) + 2] = 0ull;
        }
    }
    uint16_t* my = lst + (size_t)lane * cap;
    int cnt = 0, nang = 0;
#define NNP_TEST(k)                                                                            \
    {                                                                                          \
        const int j_ = sid[k];                                                                 \
        const T d0 = sx[4 * (k)] - xi0, d1 = sx[4 * (k) + 1] - xi1, d2 = sx[4 * (k) + 2] - xi2; \
        const T r2 = d0 * d0 + d1 * d1 + d2 * d2;                                             \
        if (act && j_ != il && (pass == 0 ? (r2 < rca2) : (r2 >= rca2 && r2 < rcr2))) {        \
            if (cnt < cap) my[cnt] = (uint16_t)j_;                                             \
            ++cnt;                                                                             \
        }                                                                                      \
    }
    {
        const int ncell = nc0 * nc1 * nc2;
        const int c0 = act ? min((int)((xi0 - lo0) * ih0), nc0 - 1) : 0;
        const int c1 = act ? min((int)((xi1 - lo1) * ih1), nc1 - 1) : 0;
        const int c2 = act ? min((int)((xi2 - lo2) * ih2), nc2 - 1) : 0;
        for (int pass = 0; pass < 2; ++pass) {
            for (int q = 0; q < S; ++q)
                for (int z = max(c2 - 1, 0); z <= min(c2 + 1, nc2 - 1); ++z)
                    for (int y = max(c1 - 1, 0); y <= min(c1 + 1, nc1 - 1); ++y)
                        for (int xx = max(c0 - 1, 0); xx <= min(c0 + 1, nc0 - 1); ++xx) {
                            const int key = q * ncell + (z * nc1 + y) * nc0 + xx;
                            for (int k = kstart[key]; k < kstart[key + 1]; ++k) NNP_TEST(k)
                        }
            if (pass == 0) nang = cnt;
        }
    }
#undef NNP_TEST
    if (act) {
        int nall = cnt;
        if (nall > cap) {
            atomicOr(flag, FLAG_CAPACITY);
            nall = cap;
            nang = nang > cap ? cap : nang;
        }
        nbr_cnt[(size_t)a0 + il] = nang | (nall << 16);
    }
    wave_sync();
    // coalesced copy of the chunk's lists
    const int na = min(kNbrChunk, n - i0);
    uint16_t* dst = nbr + ((size_t)a0 + i0) * cap;
    for (int e = lane; e < na * cap; e += 64) dst[e] = lst[e];
}

// Neighbour lists of molecules of at most cell_min atoms, one wave per
// central atom and one lane per candidate: the molecule is staged in element
// order (as k_neighbours does), each 64-candidate slice is tested at once and
// its hits are appended in order through a ballot, angular ones (r < rca) in
// a first sweep and the rest (r < rcr) in a second.  The lists equal those of
// the scanning kernel entry for entry; no lane walks the molecule serially.
// One wave: the molecule's atoms staged in stable element order (sx4: x y z
// and a spare word per atom, sid: input index of each staged atom).
template <typename T>
__device__ inline void stage_element_order(const T* tx, const int* tsp, int n, int S, T* sx4, int* sid) {
    const int lane = lane_id();
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int base = 0;
    for (int q = 0; q < S; ++q)
        for (int j0 = 0; j0 < n; j0 += 64) {
            const int j = j0 + lane;
            const int s = j < n ? tsp[j] : -1;
            const unsigned long long m = __ballot(s == q);
            if (s == q) {
                const int pos = base + __popcll(m & lt);
                sid[pos] = j;
                sx4[4 * pos + 0] = tx[3 * j + 0];
                sx4[4 * pos + 1] = tx[3 * j + 1];
                sx4[4 * pos + 2] = tx[3 * j + 2];
            }
            base += __popcll(m);
        }
}

// One wave: the neighbours of atom il within Rcr, those within Rca first,
// each run in the staged (element) order, one lane per candidate and hits
// appended through ballots; written to out and, if given, out2.  Returns
// the packed counts nang | nall << 16, clamped to cap (an overflow raises the
// capacity flag; writes stay within cap).
template <typename T>
__device__ inline int atom_neighbours(const T* sx4, const int* sid, int n, int il, T xi0, T xi1, T xi2,
                                      T rca2, T rcr2, int cap, uint16_t* out, uint16_t* out2,
                                      int32_t* __restrict__ flag) {
    const int lane = lane_id();
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int cnt = 0, nang = 0;
    for (int pass = 0; pass < 2; ++pass) {
        for (int k0 = 0; k0 < n; k0 += 64) {
            const int k = k0 + lane;
            bool hit = false;
            int j = 0;
            if (k < n) {
                j = sid[k];
                const T d0 = sx4[4 * k] - xi0, d1 = sx4[4 * k + 1] - xi1, d2 = sx4[4 * k + 2] - xi2;
                const T r2 = d0 * d0 + d1 * d1 + d2 * d2;
                hit = j != il && (pass == 0 ? (r2 < rca2) : (r2 >= rca2 && r2 < rcr2));
            }
            const unsigned long long m = __ballot(hit);
            const int pos = cnt + __popcll(m & lt);
            if (hit && pos < cap) {
                out[pos] = (uint16_t)j;
                if (out2) out2[pos] = (uint16_t)j;
            }
            cnt += __popcll(m);
        }
        if (pass == 0) nang = cnt;
    }
    int nall = cnt;
    if (nall > cap) {
        if (lane == 0) atomicOr(flag, FLAG_CAPACITY);
        nall = cap;
        nang = nang > cap ? cap : nang;
    }
    return nang | (nall << 16);
}

template <typename T>
__global__ __launch_bounds__(256) void k_nbr_pairs(int A, int S, int max_apm, int cell_min, int chunk,
                                                   int cap, T rca2, T rcr2,
                                                   const int32_t* __restrict__ mol_off,
                                                   const int32_t* __restrict__ species,
                                                   const T* __restrict__ x, T* __restrict__ F,
                                                   unsigned long long* __restrict__ Fq,
                                                   uint16_t* __restrict__ nbr,
                                                   int32_t* __restrict__ nbr_cnt,
                                                   int32_t* __restrict__ flag) {
    extern __shared__ __align__(16) char smem[];
    const int b = blockIdx.x;
    const int a0 = mol_off[b], n = mol_off[b + 1] - a0;
    if (n <= 0 || n > max_apm || n > cell_min || a0 < 0 || a0 + n > A) return;
    const int i0 = blockIdx.y * chunk;
    if (i0 >= n) return;
    const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6, nw = blockDim.x >> 6;
    LdsBump lb(smem);
    T* sx = lb.take<T>(4 * (size_t)max_apm);   // staged atoms x y z (element order)
    int* sid = lb.take<int>(max_apm);          // input index of the k-th staged atom
    T* tx = lb.take<T>(3 * (size_t)max_apm);   // input order
    int* tsp = lb.take<int>(max_apm);
    for (int t = tid; t < 3 * n; t += blockDim.x) tx[t] = x[3 * (size_t)a0 + t];
    for (int j = tid; j < n; j += blockDim.x) {
        const int s = species[a0 + j];
        tsp[j] = (s < 0 || s >= S) ? 0 : s;
    }
    __syncthreads();
    if (wave == 0) stage_element_order(tx, tsp, n, S, sx, sid);
    __syncthreads();
    const int nc = min(chunk, n - i0);
    for (int ic = wave; ic < nc; ic += nw) {
        const int il = i0 + ic;
        if (F && lane < 3) F[3 * ((size_t)a0 + il) + lane] = T(0);
        if (Fq && lane < 3) Fq[3 * ((size_t)a0 + il) + lane] = 0ull;
        const int cnt = atom_neighbours(sx, sid, n, il, tx[3 * il], tx[3 * il + 1], tx[3 * il + 2], rca2, rcr2,
                                        cap, nbr + ((size_t)a0 + il) * cap, (uint16_t*)nullptr, flag);
        if (lane == 0) nbr_cnt[(size_t)a0 + il] = cnt;
    }
}

template <typename P>
hipError_t launch_neighbours(const Shape& sh, const AevConst<typename P::T>& c,
                             const int32_t* mol_off, const int32_t* species,
                             const typename P::T* x, typename P::T* F, bool accumulate, Work<P>& w,
                             hipStream_t st, const Timer& tm) {
    typedef typename P::T T;
    // the neighbour kernels clear the force accumulators of the evaluation:
    // the integer sums when forces are summed in fixed point, else F itself
    // unless the forces accumulate onto it
    unsigned long long* Fq = nullptr;
    if (F && sh.force_fixed) {
        Fq = w.Fq;
        F = nullptr;
    } else if (accumulate) {
        F = nullptr;
    }
    // molecules up to cell_min atoms: one wave per central atom
    {
        const int small = std::min(sh.max_apm, sh.cell_min);
        dim3 grid(sh.B, (small + sh.chunk - 1) / sh.chunk);
        const size_t lds = lds_bytes<T>(4 * (size_t)sh.max_apm) + lds_bytes<int>(sh.max_apm) +
                           lds_bytes<T>(3 * (size_t)sh.max_apm) + lds_bytes<int>(sh.max_apm);
        if (lds > kMaxLds) return hipErrorInvalidValue;
        hipError_t e = ensure_lds((const void*)k_nbr_pairs<T>, lds);
        if (e != hipSuccess) return e;
        tm.b("neighbours", st);
        hipLaunchKernelGGL(k_nbr_pairs<T>, grid, dim3(256), lds, st, sh.A, sh.S, sh.max_apm, sh.cell_min,
                           sh.chunk, sh.cap_nbr, c.rca2, c.rcr2, mol_off, species, x, F, Fq, w.nbr,
                           w.nbr_cnt, w.flag);
        tm.e("neighbours", st);
        if ((e = hipGetLastError()) != hipSuccess || sh.max_apm <= sh.cell_min) return e;
    }
    // larger molecules: cutoff cells, one lane per central atom
    dim3 grid(sh.B, (sh.max_apm + kNbrChunk - 1) / kNbrChunk);
    const int nkeys = kMaxSpecies * kMaxCellsPerDim * kMaxCellsPerDim * kMaxCellsPerDim;
    const size_t lds = lds_bytes<T>(4 * (size_t)sh.max_apm) + lds_bytes<int>(sh.max_apm) +
                       lds_bytes<uint16_t>((size_t)kNbrChunk * sh.cap_nbr) +
                       lds_bytes<T>(3 * (size_t)sh.max_apm) + lds_bytes<int>(sh.max_apm) +
                       lds_bytes<int>(nkeys + 1) + lds_bytes<int>(nkeys) + lds_bytes<int>(sh.max_apm);
    if (lds > kMaxLds) return hipErrorInvalidValue;
    hipError_t e = ensure_lds((const void*)k_neighbours<T>, lds);
    if (e != hipSuccess) return e;
    tm.b("neighbours", st);
    hipLaunchKernelGGL(k_neighbours<T>, grid, dim3(64), lds, st, sh.A, sh.S, sh.max_apm,
                       sh.cell_min, sh.cap_nbr, c.rcr, c.rca2, c.rcr2, mol_off, species, x, F, Fq,
                       w.nbr, w.nbr_cnt, w.flag);
    tm.e("neighbours", st);
    return hipGetLastError();
}

// ==========================================================================
// Shared set-up of the AEV and force kernels: the molecule's coordinates and
// elements, and the chunk's neighbour counts, bucket rows and neighbour lists,
// all staged in LDS once per workgroup.
// Per-neighbour LDS record: dx dy dz r fc_r dfc_r fc_a dfc_a, padded to an
// odd number of words so that lanes reading the same field of consecutive
// records hit distinct banks (a stride of 8 words put every fourth record on
// the same bank).  The featuriser's LDS stays within a quarter of the CU's
// 160 KB on the headline shape (four workgroups per CU): odd strides for its
// pair-factor records too would cross that line.
constexpr int kNbStride = 9;

template <typename T> struct ChunkStage {
    T* sx;            // [max_apm*3]
    int* ssp;         // [max_apm]
    int* ccnt;        // [kChunk]      packed neighbour counts
    int* crow;        // [kChunk]      bucket rows
    uint16_t* clst;   // [kChunk*cap]  neighbour lists
    // lists = false: the workgroup finds its atoms' neighbours itself, so
    // neither the lists nor their counts are staged
    __device__ void take(LdsBump& lb, int max_apm, int cap, bool lists = true) {
        sx = lb.take<T>(3 * (size_t)max_apm);
        ssp = lb.take<int>(max_apm);
        ccnt = lists ? lb.take<int>(kChunk) : nullptr;
        crow = lb.take<int>(kChunk);
        clst = lists ? lb.take<uint16_t>((size_t)kChunk * cap) : nullptr;
    }
    static size_t bytes(int max_apm, int cap, bool lists = true) {
        return lds_bytes<T>(3 * (size_t)max_apm) + lds_bytes<int>(max_apm) +
               (lists ? 2 : 1) * lds_bytes<int>(kChunk) + (lists ? lds_bytes<uint16_t>((size_t)kChunk * cap) : 0);
    }
    // (zlut: species are atomic numbers; row_of_atom null: crow already set)
    __device__ void load(const T* __restrict__ x, const int32_t* __restrict__ species, int S,
                         int a0, int n, int i0, int nc, int cap,
                         const uint16_t* __restrict__ nbr, const int32_t* __restrict__ nbr_cnt,
                         const int32_t* __restrict__ row_of_atom, const int8_t* __restrict__ zlut = nullptr) {
        const int tid = threadIdx.x;
        for (int t = tid; t < 3 * n; t += blockDim.x) sx[t] = x[3 * (size_t)a0 + t];
        for (int t = tid; t < n; t += blockDim.x) {
            int s = species[a0 + t];
            if (zlut) s = (s >= 0 && s < kZLut) ? (int)zlut[s] : -1;
            ssp[t] = (s < 0 || s >= S) ? 0 : s;
        }
        for (int t = tid; t < nc; t += blockDim.x) {
            if (ccnt) ccnt[t] = nbr_cnt[(size_t)a0 + i0 + t];
            if (row_of_atom) crow[t] = row_of_atom[(size_t)a0 + i0 + t];
        }
        if (clst) {
            const uint16_t* src = nbr + ((size_t)a0 + i0) * cap;
            for (int e = tid; e < nc * cap; e += blockDim.x) clst[e] = src[e];
        }
    }
};

template <typename T>
__device__ inline void load_neighbours(const AevConst<T>& c, const T* __restrict__ sx,
                                       const int* __restrict__ ssp,
                                       const uint16_t* __restrict__ nb_list, int nang, int nall,
                                       int il, T* __restrict__ nb, int* __restrict__ nsp,
                                       int* __restrict__ nid) {
    const T xi0 = sx[3 * il], xi1 = sx[3 * il + 1], xi2 = sx[3 * il + 2];
    for (int t = lane_id(); t < nall; t += 64) {
        const int j = nb_list[t];
        const T d0 = sx[3 * j] - xi0, d1 = sx[3 * j + 1] - xi1, d2 = sx[3 * j + 2] - xi2;
        const T r = m_sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        T* e = nb + kNbStride * t;
        e[0] = d0;
        e[1] = d1;
        e[2] = d2;
        e[3] = r;
        e[4] = T(0.5) * m_cos(c.pi_rcr * r) + T(0.5);
        e[5] = -T(0.5) * c.pi_rcr * m_sin(c.pi_rcr * r);
        if (t < nang) {
            e[6] = T(0.5) * m_cos(c.pi_rca * r) + T(0.5);
            e[7] = -T(0.5) * c.pi_rca * m_sin(c.pi_rca * r);
        } else {
            e[6] = T(0);
            e[7] = T(0);
        }
        nsp[t] = ssp[j];
        nid[t] = j;
    }
}

// The record's ninth word (padding otherwise) carries its tag: neighbour
// index j << 8 | element of j, so the featuriser and force kernels keep no
// per-neighbour index arrays beside the records.
__device__ inline void put_tag(float* e, int v) { e[8] = __int_as_float(v); }
__device__ inline void put_tag(double* e, int v) { e[8] = (double)v; }
__device__ inline int tag_of(const float* e) { return __float_as_int(e[8]); }
__device__ inline int tag_of(const double* e) { return (int)e[8]; }
static_assert(kNbStride >= 9, "record tag slot");

// load_neighbours with the tag in the record instead of nsp / nid
template <typename T>
__device__ inline void load_records(const AevConst<T>& c, const T* __restrict__ sx,
                                    const int* __restrict__ ssp,
                                    const uint16_t* __restrict__ nb_list, int nang, int nall,
                                    int il, T* __restrict__ nb) {
    const T xi0 = sx[3 * il], xi1 = sx[3 * il + 1], xi2 = sx[3 * il + 2];
    for (int t = lane_id(); t < nall; t += 64) {
        const int j = nb_list[t];
        const T d0 = sx[3 * j] - xi0, d1 = sx[3 * j + 1] - xi1, d2 = sx[3 * j + 2] - xi2;
        const T r = m_sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        T* e = nb + kNbStride * t;
        e[0] = d0;
        e[1] = d1;
        e[2] = d2;
        e[3] = r;
        e[4] = T(0.5) * m_cos(c.pi_rcr * r) + T(0.5);
        e[5] = -T(0.5) * c.pi_rcr * m_sin(c.pi_rcr * r);
        if (t < nang) {
            e[6] = T(0.5) * m_cos(c.pi_rca * r) + T(0.5);
            e[7] = -T(0.5) * c.pi_rca * m_sin(c.pi_rca * r);
        } else {
            e[6] = T(0);
            e[7] = T(0);
        }
        put_tag(e, (j << 8) | ssp[j]);
    }
}

// --------------------------------------------------------------------------
// Per-atom structure of an element-sorted neighbour list.  The angular run
// (r < rca) and the radial-only run are each sorted by element, so the
// neighbours of element s form one contiguous range in each run, and the
// angular pairs {j < k} whose elements make the unordered pair (a, b) form a
// rectangle (a < b) or a triangle (a == b) of index space.  Pairs are
// numbered block by block (blocks in AEV order, i.e. by pair_index(a, b)), so
// every 32-slot angular block of the AEV is a contiguous pair range and can
// be summed by the lanes that own its slots, with no atomics.
template <typename T> struct AtomLists {
    int* aoff;   // [kMaxSpecies + 1]  angular-run start of each element
    int* roff;   // [kMaxSpecies + 1]  radial-only-run start of each element
    int* bst;    // [kMaxBlocks + 1]   first pair of each angular block
    static constexpr int kMaxBlocks = kMaxSpecies * (kMaxSpecies + 1) / 2;
    __device__ void take(LdsBump& lb) {
        aoff = lb.take<int>(kMaxSpecies + 1);
        roff = lb.take<int>(kMaxSpecies + 1);
        bst = lb.take<int>(kMaxBlocks + 1);
    }
    static constexpr size_t bytes() {
        return 2 * (((kMaxSpecies + 1) * sizeof(int) + 15) & ~size_t(15)) +
               (((kMaxBlocks + 1) * sizeof(int) + 15) & ~size_t(15));
    }
};

// elements (a, b), a <= b, of the angular block with triangular index L
__device__ inline void block_elements(int L, int S, int& a, int& b) {
    int base = 0, aa = 0;
    while (aa < S - 1 && L >= base + (S - aa)) {
        base += S - aa;
        ++aa;
    }
    a = aa;
    b = aa + (L - base);
}

// Fill aoff / roff / bst for one atom (wave-wide); sp_of(t) = element of
// neighbour t.  Returns the number of angular pairs.
template <typename T, typename SpOf>
__device__ inline int atom_lists(const AtomLists<T>& al, SpOf sp_of, int nang, int nall, int S) {
    const int lane = lane_id();
    // Both runs (angular [0, nang), radial-only [nang, nall)) are sorted by
    // element: the first neighbour of each element in a run marks where that
    // element starts; an element absent from a run starts where the next
    // present one does (or at the run's end).
    if (lane <= S) {
        al.aoff[lane] = nang;
        al.roff[lane] = nall;
    }
    wave_sync();
    for (int t = lane; t < nall; t += 64) {
        const int sp = sp_of(t);
        if (t == 0 || t == nang || sp_of(t - 1) != sp) {
            if (t < nang) al.aoff[sp] = t;
            else al.roff[sp] = t;
        }
    }
    wave_sync();
    int ao = lane <= S ? al.aoff[lane] : nang, ro = lane <= S ? al.roff[lane] : nall;
    for (int o = 1; o <= 8; o <<= 1) {   // suffix minimum over lanes 0..S
        const int va = __shfl_down(ao, o), vr = __shfl_down(ro, o);
        if (lane + o <= S) {
            ao = min(ao, va);
            ro = min(ro, vr);
        }
    }
    if (lane <= S) {
        al.aoff[lane] = ao;
        al.roff[lane] = ro;
    }
    // lane s: angular neighbours of element s (the shuffle runs on every
    // lane: a lane outside the condition would not supply its value)
    const int ao_next = __shfl_down(ao, 1);
    const int ca = lane < S ? ao_next - ao : 0;
    // angular block sizes and their prefix
    const int NB = S * (S + 1) / 2;
    int a = 0, b = 0;
    if (lane < NB) block_elements(lane, S, a, b);
    const int na = __shfl(ca, a), nb = __shfl(ca, b);
    const int cnt = lane < NB ? (a < b ? na * nb : na * (na - 1) / 2) : 0;
    int inc = cnt;
    for (int o = 1; o < 64; o <<= 1) {
        const int v = __shfl_up(inc, o);
        if (lane >= o) inc += v;
    }
    if (lane < NB) al.bst[lane + 1] = inc;
    if (lane == 0) al.bst[0] = 0;
    return __shfl(inc, NB - 1);
}

// neighbour indices (j, k) of angular pair p (block-ordered numbering)
template <typename T>
__device__ inline void pair_of(const AtomLists<T>& al, int NB, int S, int p, int& j, int& k) {
    int lo = 0;   // last block with bst[lo] <= p
    for (int step = 32; step > 0; step >>= 1)
        if (lo + step < NB && al.bst[lo + step] <= p) lo += step;
    int a, b;
    block_elements(lo, S, a, b);
    const int u = p - al.bst[lo];
    if (a < b) {
        const int nb = al.aoff[b + 1] - al.aoff[b];
        // u / nb through the float reciprocal, corrected (u < 2^16)
        int q = (int)((float)u * __builtin_amdgcn_rcpf((float)nb));
        if (q * nb > u) --q;
        if ((q + 1) * nb <= u) ++q;
        j = al.aoff[a] + q;
        k = al.aoff[b] + (u - q * nb);
    } else {
        int jj, kk;
        decode_pair(u, al.aoff[a + 1] - al.aoff[a], jj, kk);
        j = al.aoff[a] + jj;
        k = al.aoff[a] + kk;
    }
}

// Bucketing inside the featuriser, for batches of at most kPrepBlock atoms and
// molecules: the steps and results of k_bucket_one without its launch.  Every
// workgroup counts the elements of the batch's atoms per 64-atom segment
// (ballots) and forms the padded bucket offsets (prefix over the lanes of
// wave 0); it then places its own central atoms [c0, c0 + nc) (row = bucket
// start + atoms of the element in earlier segments + rank in its segment),
// keeps their rows in crow and writes their per-atom outputs.  The lead
// workgroup also writes the bucket table, the row tiles' elements, the
// padding rows and the capacity flags.  Returns false when the rows exceed
// the capacity (the rows are then not written, as the kernel leaves them).
constexpr int kBucketScratch = (kPrepBlock / 64) * kMaxSpecies + 2 * kMaxSpecies + 1 + 2 * kChunk;
__device__ inline bool bucket_in_features(const BucketFuse& bk, int S, int A, int max_apm,
                                          const int32_t* __restrict__ mol_off,
                                          const int32_t* __restrict__ species, int b, int c0, int nc,
                                          bool mine, bool lead, int* scr, int* crow,
                                          int32_t* __restrict__ flag) {
    int* segcnt = scr;                                   // [segment][element]
    int* base = segcnt + (kPrepBlock / 64) * kMaxSpecies;   // [S + 1] padded starts
    int* tot = base + kMaxSpecies + 1;                   // [S] atoms per element
    int* crank = tot + kMaxSpecies;                      // [nc] rank in its segment
    int* csp = crank + kChunk;                           // [nc] element (| 0x100: invalid)
    const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6, nw = blockDim.x >> 6;
    int A0, A1;
    const bool rng = atom_range(A, bk.B, bk.dA, mol_off, bk.sub, A0, A1);
    if (lead) {
        if (!rng && tid == 0) atomicOr(flag, FLAG_CAPACITY);
        for (int m = tid; m < bk.B; m += blockDim.x) {
            const int m0 = mol_off[m], m1 = mol_off[m + 1];
            if (m0 < A0 || m1 < m0 || m1 > A1 || m1 - m0 > max_apm) atomicOr(flag, FLAG_CAPACITY);
        }
    }
    // central atoms outside the call's range have no row (the lead has flagged them)
    mine = mine && c0 >= A0 && c0 + nc <= A1;
    const int nseg = (A1 - A0 + 63) >> 6;
    const unsigned long long lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    for (int g = wave; g < nseg; g += nw) {
        const int a = A0 + 64 * g + lane;
        int sv = -1;
        if (a < A1) {
            sv = species[a];
            if (bk.zlut) sv = (sv >= 0 && sv < kZLut) ? (int)bk.zlut[sv] : -1;
            if (sv >= S) sv = -1;
        }
        const int s = sv < 0 ? 0 : sv;   // as the bucketing kernel counts them
        for (int q = 0; q < S; ++q) {
            const unsigned long long m = __ballot(a < A1 && s == q);
            if (lane == 0) segcnt[g * kMaxSpecies + q] = __popcll(m);
            if (a < A1 && s == q && a >= c0 && a < c0 + nc) {
                crank[a - c0] = __popcll(m & lt);
                csp[a - c0] = q | (sv < 0 ? 0x100 : 0);
            }
        }
    }
    __syncthreads();
    if (wave == 0) {
        int c = 0;
        if (lane < S)
            for (int g = 0; g < nseg; ++g) c += segcnt[g * kMaxSpecies + lane];
        const int pc = ((c + bk.row_tile - 1) / bk.row_tile) * bk.row_tile;
        int incl = pc;
        for (int d = 1; d < 2 * kMaxSpecies; d <<= 1) {
            const int v = __shfl_up(incl, d);
            if (lane >= d) incl += v;
        }
        if (lane < S) tot[lane] = c;
        if (lane <= S) base[lane] = incl - pc;
        if (lead) {
            if (lane < S) bk.info->count[lane] = c;
            if (lane <= S) bk.info->off[lane] = incl - pc;
            if (lane == S) {
                int rows = incl;
                if (rows > bk.Rcap) {
                    atomicOr(flag, FLAG_CAPACITY);
                    rows = 0;
                }
                bk.info->rows = rows;
            }
        }
    }
    __syncthreads();
    const bool fits = base[S] <= bk.Rcap;
    const int rows = fits ? base[S] : 0;
    if (lead) {
        for (int t = tid; t < bk.Rcap / bk.row_tile; t += blockDim.x) {
            const int r = t * bk.row_tile;
            int sp = -1;
            if (r < rows)
                for (int q = 0; q < S; ++q)
                    if (base[q] <= r && r < base[q + 1]) sp = q;
            bk.tile_species[t] = sp;
        }
        for (int q = 0; q < S; ++q)
            for (int r = base[q] + tot[q] + tid; r < base[q + 1] && r < rows; r += blockDim.x)
                bk.atom_of_row[r] = -1;
    }
    if (!fits || !mine) return false;
    for (int ic = tid; ic < nc; ic += blockDim.x) {
        const int a = c0 + ic, s = csp[ic] & 0xff, g = (a - A0) >> 6;
        int row = base[s] + crank[ic];
        for (int g2 = 0; g2 < g; ++g2) row += segcnt[g2 * kMaxSpecies + s];
        crow[ic] = row;
        bk.row_of_atom[a] = row;
        bk.atom_of_row[row] = a;
        bk.mol_of_atom[a] = b;
        if (bk.zlut) bk.sp_out[a] = s;
        if (csp[ic] & 0x100) atomicOr(flag, FLAG_SPECIES);
    }
    __syncthreads();
    return true;
}

// --------------------------------------------------------------------------
// AEV forward.  One wave per central atom; the output row of atom a goes to
// G[row_of_atom[a]] in the GEMM operand type, optionally also to aev_out[a]
// (atom order, unpadded).  Every AEV slot is owned by one lane: radial slot
// (s, k) by lane (group s % 4, shift k) summing over the neighbours of
// element s; angular slots l and l + 16 of a block by lane l of one
// quarter-wave (the blocks meeting a 64-pair batch are dealt to the four
// quarters in turn, and a block's pairs are contiguous).  Pair factors (NA distance
// terms, NZ angle terms) are computed once per pair, 64 pairs at a time,
// into LDS.  Each slot is stored to the output row by its owner lane as soon
// as it is complete: no row is assembled in LDS, which keeps the workgroup's
// LDS small enough for more waves per CU.
template <typename P, int NZ, bool BUCKET = false>
__global__ __launch_bounds__(256, sizeof(typename P::T) == 8 ? 1 : 6) void k_aev(AevConst<typename P::T> c, int A, int max_apm,
                                             int chunk, int cap, const int32_t* __restrict__ mol_off,
                                             const int32_t* __restrict__ species,
                                             const typename P::T* __restrict__ x,
                                             const uint16_t* __restrict__ nbr,
                                             const int32_t* __restrict__ nbr_cnt,
                                             const int32_t* __restrict__ row_of_atom,
                                             typename P::TS* __restrict__ G,
                                             typename P::T* __restrict__ aev_out,
                                             NbrFuse<typename P::T> nf) {
    typedef typename P::T T;
    typedef typename P::TS TS;
    constexpr int NA = kNAZ / NZ;
    constexpr int PF = NA + NZ;
    extern __shared__ __align__(16) char smem[];
    const int b = blockIdx.x;
    const int a0 = mol_off[b], n = mol_off[b + 1] - a0;
    const int i0 = blockIdx.y * chunk;
    // with the bucketing fused in, workgroup (0, 0) also writes the batch's
    // bucket table, whether or not it has central atoms
    constexpr bool bucket = BUCKET;
    bool mine = true, lead = false;
    if constexpr (bucket) {
        mine = !(n <= 0 || n > max_apm || a0 < 0 || a0 + n > A) && i0 < n;
        lead = b == 0 && blockIdx.y == 0;
        if (!mine && !lead) return;
    } else {
        if (n <= 0 || n > max_apm || a0 < 0 || a0 + n > A) return;
        if (i0 >= n) return;
    }
    const int nc = mine ? min(chunk, n - i0) : 0;
    const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6, nw = blockDim.x >> 6;
    const int S = c.S, RL = kNR * S, NB = S * (S + 1) / 2;

    // fused: the workgroup finds its atoms' neighbour lists itself (and
    // writes them out for the force kernel) instead of reading them
    const bool fuse = nf.nbr != nullptr;
    LdsBump lb(smem);
    ChunkStage<T> cs;
    cs.take(lb, max_apm, cap, !fuse);
    if constexpr (bucket) {
        int* scr = lb.take<int>(kBucketScratch);
        if (!bucket_in_features(nf.bk, S, A, max_apm, mol_off, species, b, a0 + i0, nc, mine, lead, scr,
                                cs.crow, nf.flag))
            return;
    }
    T* nb = lb.take<T>((size_t)nw * cap * kNbStride) + (size_t)wave * cap * kNbStride;
    T* pf = lb.take<T>((size_t)nw * 64 * PF) + (size_t)wave * 64 * PF;
    T* sx4 = fuse ? lb.take<T>(4 * (size_t)max_apm) : nullptr;
    int* sid = fuse ? lb.take<int>(max_apm) : nullptr;
    uint16_t* wl = fuse ? lb.take<uint16_t>((size_t)nw * cap) + (size_t)wave * cap : nullptr;
    AtomLists<T> al;
    {
        LdsBump lw(lb.p + (size_t)wave * AtomLists<T>::bytes());
        al.take(lw);
    }
    if constexpr (bucket) cs.load(x, species, S, a0, n, i0, nc, cap, nbr, nbr_cnt, nullptr, nf.bk.zlut);
    else cs.load(x, species, S, a0, n, i0, nc, cap, nbr, nbr_cnt, row_of_atom);
    __syncthreads();
    if (fuse) {
        if (wave == 0) stage_element_order(cs.sx, cs.ssp, n, S, sx4, sid);
        __syncthreads();
    }

    // angular block sums by quarter-waves: lane (r = lane / 16, l = lane % 16)
    // owns slots l and l + 16 of the block dealt to quarter r
    const int qr = lane >> 4, ql = lane & 15;
    const int qa1 = ql / NZ, qa2 = (ql + 16) / NZ, qzl = ql % NZ;
    for (int ic = wave; ic < nc; ic += nw) {
        const int il = i0 + ic;
        int cnt;
        const uint16_t* lst;
        if (fuse) {
            // this evaluation's force accumulators, cleared as the neighbour
            // kernel clears them
            if (nf.F && lane < 3) nf.F[3 * ((size_t)a0 + il) + lane] = T(0);
            if (nf.Fq && lane < 3) nf.Fq[3 * ((size_t)a0 + il) + lane] = 0ull;
            cnt = atom_neighbours(sx4, sid, n, il, cs.sx[3 * il], cs.sx[3 * il + 1], cs.sx[3 * il + 2], nf.rca2,
                                  nf.rcr2, cap, wl, nf.nbr + ((size_t)a0 + il) * cap, nf.flag);
            if (lane == 0) nf.cnt[(size_t)a0 + il] = cnt;
            wave_sync();
            lst = wl;
        } else {
            cnt = cs.ccnt[ic];
            lst = cs.clst + (size_t)ic * cap;
        }
        const int nang = cnt & 0xffff, nall = cnt >> 16;
        load_records(c, cs.sx, cs.ssp, lst, nang, nall, il, nb);
        wave_sync();
        const int npair = atom_lists(al, [&](int t) { return tag_of(nb + kNbStride * t) & 0xff; }, nang, nall, S);
        wave_sync();
        // every slot is stored once, straight from the lane that owns it
        TS* grow = G + (size_t)cs.crow[ic] * c.Dp;
        T* arow = aev_out ? aev_out + ((size_t)a0 + il) * c.D : nullptr;
        auto put = [&](int e, T v) {
            grow[e] = Store<TS>::st(v);
            if (arow) arow[e] = v;
        };
        for (int e = c.D + lane; e < c.Dp; e += 64) grow[e] = Store<TS>::st(T(0));

        // ---- radial: lane (group g, shift k) owns slots (s, k), s = g mod 4
        {
            const int g = lane >> 4, k = lane & 15;
            const T sk = c.shf_r[k];
            for (int s = g; s < S; s += 4) {
                // two accumulators, loads of four neighbours in flight
                T acc0 = T(0), acc1 = T(0);
                for (int run = 0; run < 2; ++run) {
                    const int t1 = run ? al.roff[s + 1] : al.aoff[s + 1];
                    int t = run ? al.roff[s] : al.aoff[s];
                    for (; t + 4 <= t1; t += 4) {
                        T r[4], f[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            r[u] = nb[kNbStride * (t + u) + 3];
                            f[u] = nb[kNbStride * (t + u) + 4];
                        }
#pragma unroll
                        for (int u = 0; u < 4; u += 2) {
                            const T d0 = r[u] - sk, d1 = r[u + 1] - sk;
                            acc0 += m_exp(-c.eta_r * d0 * d0) * f[u];
                            acc1 += m_exp(-c.eta_r * d1 * d1) * f[u + 1];
                        }
                    }
                    for (; t < t1; ++t) {
                        const T d = nb[kNbStride * t + 3] - sk;
                        acc0 += m_exp(-c.eta_r * d * d) * nb[kNbStride * t + 4];
                    }
                }
                put(kNR * s + k, c.radial_pref * (acc0 + acc1));
            }
        }

        // ---- angular, 64 pairs at a time.  A block's sum is stored when its
        // last pair is in; a block that runs on into the next batch leaves its
        // partial sums in the lanes of quarter 0 (carry), which take that block
        // first in the next batch.  Blocks without pairs are stored as zeros.
        const int blo = lane < NB ? al.bst[lane] : 0, bhi = lane < NB ? al.bst[lane + 1] : 0;
        const unsigned long long filled = __ballot(lane < NB && blo < bhi);
        T carry1 = T(0), carry2 = T(0);
        int carry_blk = -1;
        for (int p0 = 0; p0 < npair; p0 += 64) {
            const int nbat = min(64, npair - p0);
            if (lane < nbat) {
                int j, k;
                pair_of(al, NB, S, p0 + lane, j, k);
                const T* ej = nb + kNbStride * j;
                const T* ek = nb + kNbStride * k;
                const T rj = ej[3], rk = ek[3];
                T cs_ = (ej[0] * ek[0] + ej[1] * ek[1] + ej[2] * ek[2]) * m_rcp(rj * rk);
                cs_ = cs_ > T(1) ? T(1) : (cs_ < T(-1) ? T(-1) : cs_);
                const T cp = c.angle_scale * cs_;
                const T sn = m_sqrt(T(1) - cp * cp);
                const T fcc = ej[6] * ek[6];
                const T rm = T(0.5) * (rj + rk);
                T* f = pf + PF * lane;
#pragma unroll
                for (int a = 0; a < NA; ++a) {
                    const T d = rm - c.shf_a[a];
                    f[a] = m_exp(-c.eta_a * d * d) * fcc;
                }
#pragma unroll
                for (int z = 0; z < NZ; ++z) {
                    const T cz = cp * c.cos_z[z] + sn * c.sin_z[z];
                    f[NA + z] = T(2) * m_powu(T(0.5) * (T(1) + cz), c.zeta);
                }
            }
            wave_sync();
            // blocks meeting this batch, taken four at a time, one per
            // quarter-wave, each quarter summing its block's pairs in order
            // (two pairs' factors in flight)
            const int pe_ = p0 + nbat;
            const unsigned long long live = __ballot(lane < NB && blo < bhi && blo < pe_ && bhi > p0);
            const unsigned long long goes_on = __ballot(lane < NB && blo < bhi && blo < pe_ && bhi > pe_);
            T nc1 = T(0), nc2 = T(0);
            for (unsigned long long mset = live; mset;) {
                int bq[4], lq[4], hq[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    bq[r] = mset ? __builtin_ctzll(mset) : -1;
                    lq[r] = bq[r] >= 0 ? __builtin_amdgcn_readlane(blo, bq[r]) : 0;
                    hq[r] = bq[r] >= 0 ? __builtin_amdgcn_readlane(bhi, bq[r]) : 0;
                    mset &= mset - 1;
                }
                const int bl = qr == 0 ? bq[0] : (qr == 1 ? bq[1] : (qr == 2 ? bq[2] : bq[3]));
                const int lo = qr == 0 ? lq[0] : (qr == 1 ? lq[1] : (qr == 2 ? lq[2] : lq[3]));
                const int hi = qr == 0 ? hq[0] : (qr == 1 ? hq[1] : (qr == 2 ? hq[2] : hq[3]));
                const int s0 = bl < 0 ? 0 : max(lo, p0) - p0;
                const int e0 = bl < 0 ? 0 : min(hi, pe_) - p0;
                T a1 = T(0), a2 = T(0), b1 = T(0), b2 = T(0);
                int p = s0;
                for (; p + 2 <= e0; p += 2) {
                    const T* f0 = pf + PF * p;
                    const T* f1 = f0 + PF;
                    const T z0 = f0[NA + qzl], z1 = f1[NA + qzl];
                    const T x1 = f0[qa1], x2 = f0[qa2], y1 = f1[qa1], y2 = f1[qa2];
                    a1 += x1 * z0;
                    a2 += x2 * z0;
                    b1 += y1 * z1;
                    b2 += y2 * z1;
                }
                if (p < e0) {
                    const T* f0 = pf + PF * p;
                    const T z0 = f0[NA + qzl];
                    a1 += f0[qa1] * z0;
                    a2 += f0[qa2] * z0;
                }
                T v1 = a1 + b1, v2 = a2 + b2;
                if (bl == carry_blk) {
                    v1 += carry1;
                    v2 += carry2;
                }
                if (s0 < e0) {
                    if (hi > pe_) {
                        nc1 = v1;
                        nc2 = v2;
                    } else {
                        put(RL + kNAZ * bl + ql, v1);
                        put(RL + kNAZ * bl + ql + 16, v2);
                    }
                }
            }
            if (goes_on) {
                // the continuing block is the batch's last; its quarter is its
                // rank among the batch's blocks, mod 4
                const int cb = __builtin_ctzll(goes_on);
                const int qc = __popcll(live & ((1ull << cb) - 1)) & 3;
                carry1 = __shfl(nc1, ql + 16 * qc);
                carry2 = __shfl(nc2, ql + 16 * qc);
                carry_blk = cb;
            } else {
                carry_blk = -1;
            }
            wave_sync();
        }
        // blocks without pairs: zeros in 16-byte pieces, a few lanes per block
        {
            constexpr int VP = 16 / (int)sizeof(TS), PPB = kNAZ / VP, BPP = 64 / PPB;
            const int pc = lane % PPB;
            for (int b0 = 0; b0 < NB; b0 += BPP) {
                const int zb = b0 + lane / PPB;
                if (zb < NB && !((filled >> zb) & 1ull))
                    *(uint4*)(grow + RL + kNAZ * zb + VP * pc) = make_uint4(0u, 0u, 0u, 0u);
            }
            if (arow)
                for (int e = lane; e < NB * kNAZ; e += 64)
                    if (!((filled >> (e / kNAZ)) & 1ull)) arow[RL + e] = T(0);
        }
    }
}

template <typename T>
static size_t aev_lds(int max_apm, int cap, int Dp, int NZ, int nw, bool fuse = false, bool bucket = false) {
    const int PF = kNAZ / NZ + NZ;
    (void)Dp;
    return ChunkStage<T>::bytes(max_apm, cap, !fuse) + (bucket ? lds_bytes<int>(kBucketScratch) : 0) +
           lds_bytes<T>((size_t)nw * cap * kNbStride) +
           lds_bytes<T>((size_t)nw * 64 * PF) +
           (fuse ? lds_bytes<T>(4 * (size_t)max_apm) + lds_bytes<int>(max_apm) +
                       lds_bytes<uint16_t>((size_t)nw * cap)
                 : 0) +
           (size_t)nw * AtomLists<T>::bytes();
}

template <typename P>
hipError_t launch_aev(const Shape& sh, const AevConst<typename P::T>& c, const int32_t* mol_off,
                      const int32_t* species, const typename P::T* x, Work<P>& w,
                      typename P::T* aev_out, hipStream_t st, const Timer& tm,
                      const NbrFuse<typename P::T>& nf) {
    typedef typename P::T T;
    dim3 grid(sh.B, (sh.max_apm + sh.chunk - 1) / sh.chunk);
    int nw = kWaves;
    const bool fuse = nf.nbr != nullptr, bucket = nf.bk.info != nullptr;
    size_t lds = aev_lds<T>(sh.max_apm, sh.cap_nbr, c.Dp, c.nZ, nw, fuse, bucket);
    while (lds > kMaxLds && nw > 1) lds = aev_lds<T>(sh.max_apm, sh.cap_nbr, c.Dp, c.nZ, nw /= 2, fuse, bucket);
    if (lds > kMaxLds) return hipErrorInvalidValue;
    auto kern = bucket ? (c.nZ == 4 ? k_aev<P, 4, true> : k_aev<P, 8, true>)
                       : (c.nZ == 4 ? k_aev<P, 4> : k_aev<P, 8>);
    hipError_t e = ensure_lds((const void*)kern, lds);
    if (e != hipSuccess) return e;
    tm.b("aev", st);
    hipLaunchKernelGGL(kern, grid, dim3(64 * nw), lds, st, c, sh.A, sh.max_apm, sh.chunk, sh.cap_nbr,
                       mol_off, species, x, w.nbr, w.nbr_cnt, w.row_of_atom, w.G, aev_out, nf);
    tm.e("aev", st);
    return hipGetLastError();
}

// Neighbour lists and AEV rows.  Small batches (up to kFuseAtoms atoms, all
// molecules within the all-pairs neighbour search) take one fused launch:
// there the launch and the list round trip are a visible part of the
// latency.  Large batches measured no faster fused (the search is the same
// work inside the featuriser's waves), so they keep the neighbour kernels.
// The force accumulators are cleared as launch_neighbours clears them.
constexpr int kFuseAtoms = 4096;
template <typename P>
hipError_t launch_features(const Shape& sh, const AevConst<typename P::T>& c, const int32_t* mol_off,
                           const int32_t* species, const typename P::T* x, typename P::T* F,
                           bool accumulate, Work<P>& w, typename P::T* aev_out, hipStream_t st,
                           const Timer& tm) {
    if (sh.max_apm > sh.cell_min || sh.A > kFuseAtoms) {
        hipError_t e = launch_neighbours<P>(sh, c, mol_off, species, x, F, accumulate, w, st, tm);
        if (e != hipSuccess) return e;
        return launch_aev<P>(sh, c, mol_off, species, x, w, aev_out, st, tm, NbrFuse<typename P::T>());
    }
    NbrFuse<typename P::T> nf;
    nf.rca2 = c.rca2;
    nf.rcr2 = c.rcr2;
    nf.F = (F && !sh.force_fixed && !accumulate) ? F : nullptr;
    nf.Fq = (F && sh.force_fixed) ? w.Fq : nullptr;
    nf.nbr = w.nbr;
    nf.cnt = w.nbr_cnt;
    nf.flag = w.flag;
    return launch_aev<P>(sh, c, mol_off, species, x, w, aev_out, st, tm, nf);
}

// Bucketing and featurisation.  A batch that fits one bucketing workgroup and
// takes the fused neighbour search is bucketed inside the featuriser (one
// launch for all three steps: on a single small molecule each dependent
// launch is a visible part of the latency); otherwise the bucketing kernels
// run first.
template <typename P>
hipError_t launch_prep_features(const Shape& sh, const AevConst<typename P::T>& c, const int32_t* mol_off,
                                const int32_t* species, const typename P::T* x, typename P::T* F,
                                bool accumulate, Work<P>& w, typename P::T* aev_out, hipStream_t st,
                                const Timer& tm) {
    const bool small = sh.A > 0 && std::max(sh.A, sh.B) <= kPrepBlock && sh.max_apm <= sh.cell_min &&
                       sh.A <= kFuseAtoms;
    if (!small) {
        hipError_t e = launch_prep<P>(sh, mol_off, species, w, st, tm);
        if (e != hipSuccess) return e;
        if (sh.A == 0) return hipSuccess;
        return launch_features<P>(sh, c, mol_off, w.zlut ? w.sp : species, x, F, accumulate, w, aev_out, st, tm);
    }
    NbrFuse<typename P::T> nf;
    nf.rca2 = c.rca2;
    nf.rcr2 = c.rcr2;
    nf.F = (F && !sh.force_fixed && !accumulate) ? F : nullptr;
    nf.Fq = (F && sh.force_fixed) ? w.Fq : nullptr;
    nf.nbr = w.nbr;
    nf.cnt = w.nbr_cnt;
    nf.flag = w.flag;
    BucketFuse& bk = nf.bk;
    bk.zlut = w.zlut;
    bk.sp_out = w.sp;
    bk.mol_of_atom = w.mol_of_atom;
    bk.row_of_atom = w.row_of_atom;
    bk.atom_of_row = w.atom_of_row;
    bk.tile_species = w.tile_species;
    bk.info = w.info;
    bk.dA = sh.dev_counts ? w.dcnt + 1 : nullptr;
    bk.B = sh.B;
    bk.row_tile = sh.row_tile;
    bk.Rcap = sh.Rcap;
    bk.sub = sh.sub;
    return launch_aev<P>(sh, c, mol_off, species, x, w, aev_out, st, tm, nf);
}

// --------------------------------------------------------------------------
// AEV tangent (JVP): Gdot_i = sum_j dG_i/dx_j . v_j for a coordinate tangent
// v (the force-loss cotangent of training), rows written to Gd in bucket
// order.  Same structure as the forward: per pair the distance factors P_a,
// Q_a and the angle factors fz_z, dfz_z/dc are formed once, and
//   Gdot[a, z] += fz_z P_a + dfz_z Q_a,
//   P_a = A'_a rmdot F + A_a Fdot,  Q_a = A_a F cdot,
// with A_a the distance Gaussian, F = fc_j fc_k and the dotted quantities
// their rates along v.
template <typename P, int NZ>
__global__ __launch_bounds__(256) void k_aev_jvp(AevConst<typename P::T> c, int A, int max_apm,
                                                 int chunk, int cap, const int32_t* __restrict__ mol_off,
                                                 const int32_t* __restrict__ species,
                                                 const typename P::T* __restrict__ x,
                                                 const typename P::T* __restrict__ v,
                                                 const uint16_t* __restrict__ nbr,
                                                 const int32_t* __restrict__ nbr_cnt,
                                                 const int32_t* __restrict__ row_of_atom,
                                                 typename P::TS* __restrict__ Gd) {
    typedef typename P::T T;
    typedef typename P::TS TS;
    constexpr int NA = kNAZ / NZ;
    constexpr int PF = 2 * NA + 2 * NZ;       // P[NA] Q[NA] fz[NZ] dfz[NZ]
    constexpr int TS_ = 4;                     // per neighbour: v_j - v_i (3), rdot
    extern __shared__ __align__(16) char smem[];
    const int b = blockIdx.x;
    const int a0 = mol_off[b], n = mol_off[b + 1] - a0;
    if (n <= 0 || n > max_apm || a0 < 0 || a0 + n > A) return;
    const int i0 = blockIdx.y * chunk;
    if (i0 >= n) return;
    const int nc = min(chunk, n - i0);
    const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6, nw = blockDim.x >> 6;
    const int S = c.S, RL = kNR * S;

    LdsBump lb(smem);
    ChunkStage<T> cs;
    cs.take(lb, max_apm, cap);
    T* sv = lb.take<T>(3 * (size_t)max_apm);
    T* nb = lb.take<T>((size_t)nw * cap * kNbStride) + (size_t)wave * cap * kNbStride;
    T* nt = lb.take<T>((size_t)nw * cap * TS_) + (size_t)wave * cap * TS_;
    int* nsp = lb.take<int>((size_t)nw * cap) + (size_t)wave * cap;
    int* nid = lb.take<int>((size_t)nw * cap) + (size_t)wave * cap;
    T* row = lb.take<T>((size_t)nw * c.Dp) + (size_t)wave * c.Dp;
    T* pf = lb.take<T>((size_t)nw * 64 * PF) + (size_t)wave * 64 * PF;
    int* pb = lb.take<int>((size_t)nw * 64) + (size_t)wave * 64;
    cs.load(x, species, S, a0, n, i0, nc, cap, nbr, nbr_cnt, row_of_atom);
    for (int t = tid; t < 3 * n; t += blockDim.x) sv[t] = v[3 * (size_t)a0 + t];
    __syncthreads();

    for (int ic = wave; ic < nc; ic += nw) {
        const int il = i0 + ic;
        const int cnt = cs.ccnt[ic];
        const int nang = cnt & 0xffff, nall = cnt >> 16;
        load_neighbours(c, cs.sx, cs.ssp, cs.clst + (size_t)ic * cap, nang, nall, il, nb, nsp, nid);
        wave_sync();
        for (int t = lane; t < nall; t += 64) {
            const int j = nid[t];
            const T* e = nb + kNbStride * t;
            const T ir = m_rcp(e[3]);
            const T w0 = sv[3 * j] - sv[3 * il], w1 = sv[3 * j + 1] - sv[3 * il + 1],
                    w2 = sv[3 * j + 2] - sv[3 * il + 2];
            nt[TS_ * t + 0] = w0;
            nt[TS_ * t + 1] = w1;
            nt[TS_ * t + 2] = w2;
            nt[TS_ * t + 3] = (e[0] * w0 + e[1] * w1 + e[2] * w2) * ir;   // rdot = u . (v_j - v_i)
        }
        for (int e = lane; e < c.Dp; e += 64) row[e] = T(0);
        wave_sync();

        // ---- radial: d/dt of pref exp(-eta (r - s_k)^2) fc(r) = (d term/dr) rdot
        {
            const int g = lane >> 4, k = lane & 15;
            const T sk = c.shf_r[k];
            T acc = T(0);
            int cur = -1;
            for (int t = g; t < nall; t += 4) {
                const int sp = nsp[t];
                if (sp != cur) {
                    if (cur >= 0) lds_add(row + kNR * cur + k, acc);
                    acc = T(0);
                    cur = sp;
                }
                const T* e = nb + kNbStride * t;
                const T d = e[3] - sk;
                const T ex = c.radial_pref * m_exp(-c.eta_r * d * d);
                acc += ex * (T(-2) * c.eta_r * d * e[4] + e[5]) * nt[TS_ * t + 3];
            }
            if (cur >= 0) lds_add(row + kNR * cur + k, acc);
        }

        // ---- angular
        const int npair = nang * (nang - 1) / 2;
        const int h = lane >> 5, q = lane & 31, qa = q / NZ, qz = q % NZ;
        T acc = T(0);
        int cur = -1;
        for (int p0 = 0; p0 < npair; p0 += 64) {
            const int nbat = min(64, npair - p0);
            if (lane < nbat) {
                int j, k;
                decode_pair(p0 + lane, nang, j, k);
                const T* ej = nb + kNbStride * j;
                const T* ek = nb + kNbStride * k;
                const T rj = ej[3], rk = ek[3];
                const T ij = m_rcp(rj), ik = m_rcp(rk);
                const T uj0 = ej[0] * ij, uj1 = ej[1] * ij, uj2 = ej[2] * ij;
                const T uk0 = ek[0] * ik, uk1 = ek[1] * ik, uk2 = ek[2] * ik;
                T cs_ = uj0 * uk0 + uj1 * uk1 + uj2 * uk2;
                cs_ = cs_ > T(1) ? T(1) : (cs_ < T(-1) ? T(-1) : cs_);
                const T* tj = nt + TS_ * j;
                const T* tk = nt + TS_ * k;
                const T rjd = tj[3], rkd = tk[3];
                // cdot = ((u_k - c u_j)/r_j).(v_j - v_i) + ((u_j - c u_k)/r_k).(v_k - v_i)
                const T cdot = ((uk0 - cs_ * uj0) * tj[0] + (uk1 - cs_ * uj1) * tj[1] +
                                (uk2 - cs_ * uj2) * tj[2]) * ij +
                               ((uj0 - cs_ * uk0) * tk[0] + (uj1 - cs_ * uk1) * tk[1] +
                                (uj2 - cs_ * uk2) * tk[2]) * ik;
                const T cp = c.angle_scale * cs_;
                const T sn = m_sqrt(T(1) - cp * cp);
                const T F = ej[6] * ek[6];
                const T Fd = ej[7] * ek[6] * rjd + ej[6] * ek[7] * rkd;
                const T rm = T(0.5) * (rj + rk), rmd = T(0.5) * (rjd + rkd);
                T* f = pf + PF * lane;
#pragma unroll
                for (int a = 0; a < NA; ++a) {
                    const T d = rm - c.shf_a[a];
                    const T Aa = m_exp(-c.eta_a * d * d);
                    f[a] = T(-2) * c.eta_a * d * Aa * rmd * F + Aa * Fd;   // P_a
                    f[NA + a] = Aa * F * cdot;                            // Q_a
                }
#pragma unroll
                for (int z = 0; z < NZ; ++z) {
                    const T cz = cp * c.cos_z[z] + sn * c.sin_z[z];
                    const T hh = T(0.5) * (T(1) + cz);
                    const T hp = m_powu(hh, c.zeta - T(1));
                    f[2 * NA + z] = T(2) * hp * hh;
                    f[2 * NA + NZ + z] = c.zeta * hp * c.angle_scale *
                                         (c.cos_z[z] - cp * c.sin_z[z] * m_rcp(sn));
                }
                pb[lane] = RL + kNAZ * pair_index(nsp[j], nsp[k], S);
            }
            wave_sync();
            for (int t = h; t < nbat; t += 2) {
                const int blk = pb[t];
                if (blk != cur) {
                    if (cur >= 0) lds_add(row + cur + q, acc);
                    acc = T(0);
                    cur = blk;
                }
                const T* f = pf + PF * t;
                acc += f[2 * NA + qz] * f[qa] + f[2 * NA + NZ + qz] * f[NA + qa];
            }
            wave_sync();
        }
        if (cur >= 0) lds_add(row + cur + q, acc);
        wave_sync();
        const size_t grow = (size_t)cs.crow[ic];
        for (int e = lane; e < c.Dp; e += 64) Gd[grow * c.Dp + e] = Store<TS>::st(row[e]);
        wave_sync();
    }
}

template <typename T>
static size_t jvp_lds(int max_apm, int cap, int Dp, int NZ, int nw) {
    const int PF = 2 * (kNAZ / NZ) + 2 * NZ;
    return ChunkStage<T>::bytes(max_apm, cap) + lds_bytes<T>(3 * (size_t)max_apm) +
           lds_bytes<T>((size_t)nw * cap * kNbStride) + lds_bytes<T>((size_t)nw * cap * 4) +
           2 * lds_bytes<int>((size_t)nw * cap) + lds_bytes<T>((size_t)nw * Dp) +
           lds_bytes<T>((size_t)nw * 64 * PF) + lds_bytes<int>((size_t)nw * 64);
}

template <typename P>
hipError_t launch_aev_jvp(const Shape& sh, const AevConst<typename P::T>& c,
                          const int32_t* mol_off, const int32_t* species,
                          const typename P::T* x, const typename P::T* v, Work<P>& w,
                          typename P::TS* Gd, hipStream_t st, const Timer& tm) {
    typedef typename P::T T;
    dim3 grid(sh.B, (sh.max_apm + sh.chunk - 1) / sh.chunk);
    int nw = kWaves;
    size_t lds = jvp_lds<T>(sh.max_apm, sh.cap_nbr, c.Dp, c.nZ, nw);
    while (lds > kMaxLds && nw > 1) lds = jvp_lds<T>(sh.max_apm, sh.cap_nbr, c.Dp, c.nZ, nw /= 2);
    if (lds > kMaxLds) return hipErrorInvalidValue;
    auto kern = c.nZ == 4 ? k_aev_jvp<P, 4> : k_aev_jvp<P, 8>;
    hipError_t e = ensure_lds((const void*)kern, lds);
    if (e != hipSuccess) return e;
    tm.b("aev_jvp", st);
    hipLaunchKernelGGL(kern, grid, dim3(64 * nw), lds, st, c, sh.A, sh.max_apm, sh.chunk, sh.cap_nbr,
                       mol_off, species, x, v, w.nbr, w.nbr_cnt, w.row_of_atom, Gd);
    tm.e("aev_jvp", st);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// AEV backward: dE/dx contracted from dE/dAEV rows (dG, already scaled to
// energy units), forces F = -dE/dx accumulated per molecule in LDS and added
// to F (zeroed by the neighbour kernel) once per workgroup.
// LDS stride of one element-pair block of dG: 16-byte aligned, and 9 16-byte
// granules apart (mod the 16 granules of the banks), so lanes reading the same
// offset of different blocks spread over the banks
constexpr int kBlkPad = kNAZ + 4;

// four consecutive values of an LDS row (16-byte aligned)
__device__ inline void ld4(const float* p, float v[4]) {
    const float4 q = *(const float4*)p;
    v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
}
__device__ inline void ld4(const double* p, double v[4]) {
    const double2 a = *(const double2*)p, b = *(const double2*)(p + 2);
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
}
// four consecutive dE/dAEV values from global memory in their storage type
__device__ inline void ldg4(const float* p, float v[4]) { ld4(p, v); }
__device__ inline void ldg4(const double* p, double v[4]) { ld4(p, v); }
__device__ inline void ldg4(const bf16_t* p, float v[4]) {
    const uint2 q = *(const uint2*)p;
    v[0] = __uint_as_float(q.x << 16); v[1] = __uint_as_float(q.x & 0xffff0000u);
    v[2] = __uint_as_float(q.y << 16); v[3] = __uint_as_float(q.y & 0xffff0000u);
}
__device__ inline void st4(float* p, const float v[4]) { *(float4*)p = make_float4(v[0], v[1], v[2], v[3]); }
__device__ inline void st4(double* p, const double v[4]) {
    *(double2*)p = make_double2(v[0], v[1]);
    *(double2*)(p + 2) = make_double2(v[2], v[3]);
}

// Force accumulators.  Floating point: LDS and global atomic adds, whose
// order (and so the last bits of F) varies from run to run.  Fixed point:
// every contribution is scaled by 2^32 and rounded to a 64-bit integer
// (exact for FP32 contributions above 2^-9 in magnitude), and integer
// addition is associative, so the sums are bitwise the same whatever the
// order; the energy kernel turns them back into F.
// Energy of molecule b summed by one wave in a fixed order (atoms strided
// over the lanes, then a shuffle tree): the per-row partials of every model
// plus the output bias, the ensemble mean times the energy scale, plus the
// self-energies.
template <typename P>
__device__ inline double molecule_energy(int a0, int a1, int M, int NT, double scale,
                                         const int32_t* __restrict__ species, int S,
                                         const int32_t* __restrict__ row_of_atom,
                                         const typename P::TA* __restrict__ Epart,
                                         const typename P::TA* __restrict__ b4,
                                         const double* __restrict__ sae) {
    const int lane = lane_id();
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
        acc += scale * (e / M) + sae[s];
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    return (a1 > a0) ? acc : 0.0;
}

template <typename T, bool FIXED> struct ForceAcc;
template <typename T> struct ForceAcc<T, false> {
    typedef T V;
    __device__ static void add(V* p, T v) { lds_add(p, v); }
    __device__ static void flush(V v, T* F, unsigned long long*, size_t i) {
        if (v != V(0)) gbl_add(&F[i], v);
    }
};
constexpr double kForceFix = 4294967296.0;   // 2^32
__device__ inline long long to_fixed(float v) { return __float2ll_rn(v * 4294967296.0f); }
__device__ inline long long to_fixed(double v) { return __double2ll_rn(v * kForceFix); }
template <typename T> struct ForceAcc<T, true> {
    typedef unsigned long long V;
    __device__ static void add(V* p, T v) { atomicAdd(p, (unsigned long long)to_fixed(v)); }
    __device__ static void flush(V v, T*, unsigned long long* Fq, size_t i) {
        if (v != 0ull) atomicAdd(&Fq[i], v);
    }
};

template <typename P, int NZ, bool FIXED, bool GD>
__global__ __launch_bounds__(256, sizeof(typename P::T) == 8 ? 1 : 6) void k_forces(AevConst<typename P::T> c, int A, int max_apm,
                                                int chunk, int cap, const int32_t* __restrict__ mol_off,
                                                const int32_t* __restrict__ species,
                                                const typename P::T* __restrict__ x,
                                                const uint16_t* __restrict__ nbr,
                                                const int32_t* __restrict__ nbr_cnt,
                                                const int32_t* __restrict__ row_of_atom,
                                                const typename P::TG* __restrict__ dG,
                                                typename P::T* __restrict__ F,
                                                unsigned long long* __restrict__ Fq,
                                                EnergyArgs<P> ea) {
    typedef typename P::T T;
    typedef typename P::TA TA;
    typedef typename P::TG TG;
    typedef ForceAcc<T, FIXED> Acc;
    typedef typename Acc::V V;
    constexpr int NA = kNAZ / NZ;
    extern __shared__ __align__(16) char smem[];
    const int b = blockIdx.x;
    const int a0 = mol_off[b], n = mol_off[b + 1] - a0;
    // the molecule's energy (as k_energy computes it), by the first wave of
    // its first workgroup, ahead of the force work
    if (ea.E && blockIdx.y == 0 && threadIdx.x < 64 && b < ea.B && !(ea.dcnt && b >= ea.dcnt[0])) {
        const bool ok = !(a0 < 0 || n < 0 || a0 + n > A);
        const double v = molecule_energy<P>(ok ? a0 : 0, ok ? a0 + n : 0, ea.M, ea.NT, ea.scale, species,
                                            c.S, row_of_atom, ea.Epart, ea.b4, ea.sae);
        if (threadIdx.x == 0) ea.E[b] = ea.accumulate ? ea.E[b] + v : v;
    }
    if (n <= 0 || n > max_apm || a0 < 0 || a0 + n > A) return;
    const int i0 = blockIdx.y * chunk;
    if (i0 >= n) return;
    const int nc = min(chunk, n - i0);
    const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6, nw = blockDim.x >> 6;
    const int S = c.S, RL = kNR * S, NB = S * (S + 1) / 2;
    const int GL = RL + kBlkPad * NB;

    LdsBump lb(smem);
    ChunkStage<T> cs;
    cs.take(lb, max_apm, cap);
    V* sF = lb.take<V>(3 * (size_t)max_apm);
    T* nb = lb.take<T>((size_t)nw * cap * kNbStride) + (size_t)wave * cap * kNbStride;
    T* pg = lb.take<T>((size_t)nw * 64 * 6) + (size_t)wave * 64 * 6;   // a batch's pair forces
    // the atom's dE/dAEV row: staged in LDS (blocks kBlkPad apart), or read
    // straight from global memory (GD: L1/L2 hits, the LDS left to the
    // force sums)
    T* g = GD ? nullptr : lb.take<T>((size_t)nw * GL) + (size_t)wave * GL;
    constexpr int BS = GD ? kNAZ : kBlkPad;

    cs.load(x, species, S, a0, n, i0, nc, cap, nbr, nbr_cnt, row_of_atom);
    for (int t = tid; t < 3 * n; t += blockDim.x) sF[t] = V(0);
    __syncthreads();
    for (int ic = wave; ic < nc; ic += nw) {
        const int il = i0 + ic;
        const int cnt = cs.ccnt[ic];
        const int nang = cnt & 0xffff, nall = cnt >> 16;
        const TG* gsrc = dG + (size_t)cs.crow[ic] * c.Dp;
        // the atom's dE/dAEV row: 16 values per lane and load, all in flight
        // before the first use; groups of 16 never straddle a block
        if constexpr (!GD) {
            const TG* src = dG + (size_t)cs.crow[ic] * c.Dp;
            TA v[2][16];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int e = 16 * (lane + 64 * u);
#pragma unroll
                for (int q4 = 0; q4 < 4; ++q4)
                    if (e < c.D) ldg4(src + e + 4 * q4, &v[u][4 * q4]);
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int e = 16 * (lane + 64 * u);
                if (e < c.D) {
                    const int le = e < RL ? e : RL + kBlkPad * ((e - RL) / kNAZ) + (e - RL) % kNAZ;
                    T w[16];
#pragma unroll
                    for (int q = 0; q < 16; ++q) w[q] = (T)v[u][q];
#pragma unroll
                    for (int q4 = 0; q4 < 4; ++q4) st4(g + le + 4 * q4, &w[4 * q4]);
                }
            }
        }
        load_records(c, cs.sx, cs.ssp, cs.clst + (size_t)ic * cap, nang, nall, il, nb);
        wave_sync();
        T fi0 = 0, fi1 = 0, fi2 = 0;   // force on the central atom, per lane
        // radial: lane per (neighbour, group of 4 shifts)
        for (int it = lane; it < ((4 * nall + 63) & ~63); it += 64) {
            const bool act = it < 4 * nall;
            const int t = act ? (it >> 2) : 0, q = it & 3;
            T dEdr = 0;
            if (act) {
                const T* e = nb + kNbStride * t;
                const T r = e[3], fc = e[4], dfc = e[5];
                const int st = tag_of(e) & 0xff;
                T gg[4];
                if constexpr (GD) {
                    TA ga[4];
                    ldg4(gsrc + kNR * st + 4 * q, ga);
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) gg[kk] = (T)ga[kk];
                } else {
                    ld4(g + kNR * st + 4 * q, gg);
                }
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    const T d = r - c.shf_r[4 * q + kk];
                    const T ex = c.radial_pref * m_exp(-c.eta_r * d * d);
                    dEdr += gg[kk] * ex * (T(-2) * c.eta_r * d * fc + dfc);
                }
            }
            // the four shift groups of one neighbour sit in adjacent lanes
            dEdr += __shfl_xor(dEdr, 1);
            dEdr += __shfl_xor(dEdr, 2);
            if (act && q == 0) {
                const T* e = nb + kNbStride * t;
                const T inv = m_rcp(e[3]);
                const T u0 = e[0] * inv, u1 = e[1] * inv, u2 = e[2] * inv;
                const int j = tag_of(e) >> 8;
                // dE/dx_j = dEdr u, dE/dx_i = -dEdr u;  F = -dE/dx
                Acc::add(&sF[3 * j + 0], -dEdr * u0);
                Acc::add(&sF[3 * j + 1], -dEdr * u1);
                Acc::add(&sF[3 * j + 2], -dEdr * u2);
                fi0 += dEdr * u0;
                fi1 += dEdr * u1;
                fi2 += dEdr * u2;
            }
        }
        // angular: lane per neighbour pair, pairs in rotation order, 64 at a
        // time.  A pair's forces on its atoms j and k go to LDS with plain
        // stores; then lane (t, c) sums component c of neighbour t over the
        // batch's pairs that hold t and makes one add to the molecule's sums
        // (LDS atomic adds cost far more than stores and reads on gfx950).
        const int npair = nang * (nang - 1) / 2;
        const int full = nang * ((nang - 1) >> 1), D = (nang - 1) >> 1, half = nang >> 1;
        for (int P0 = 0; P0 < npair; P0 += 64) {
          const int p = P0 + lane, nbat = min(64, npair - P0);
          if (p < npair) {
            int j, k;
            decode_pair_rot(p, nang, j, k);
            const T* ej = nb + kNbStride * j;
            const T* ek = nb + kNbStride * k;
            const T rj = ej[3], rk = ek[3];
            const T ij = m_rcp(rj), ik = m_rcp(rk);
            const T uj0 = ej[0] * ij, uj1 = ej[1] * ij, uj2 = ej[2] * ij;
            const T uk0 = ek[0] * ik, uk1 = ek[1] * ik, uk2 = ek[2] * ik;
            T cs_ = uj0 * uk0 + uj1 * uk1 + uj2 * uk2;
            cs_ = cs_ > T(1) ? T(1) : (cs_ < T(-1) ? T(-1) : cs_);
            const T cp = c.angle_scale * cs_;
            const T sn = m_sqrt(T(1) - cp * cp);
            const T fcj = ej[6], fck = ek[6], dfcj = ej[7], dfck = ek[7];
            const T fcc = fcj * fck;
            const T rm = T(0.5) * (rj + rk);
            const int tj = tag_of(ej), tk = tag_of(ek);
            const int pb = RL + BS * pair_index(tj & 0xff, tk & 0xff, S);
            const T* gb = GD ? nullptr : g + pb;
            T fz[NZ], dfz[NZ];
#pragma unroll
            for (int z = 0; z < NZ; ++z) {
                const T cz = cp * c.cos_z[z] + sn * c.sin_z[z];
                const T hh = T(0.5) * (T(1) + cz);
                const T hp = m_powu(hh, c.zeta - T(1));
                fz[z] = T(2) * hp * hh;
                // d cos(theta'-t)/dc = s (cos t - c' sin t / sqrt(1 - c'^2))
                const T dcz = c.angle_scale * (c.cos_z[z] - cp * c.sin_z[z] * m_rcp(sn));
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
                for (int z4 = 0; z4 < NZ; z4 += 4) {
                    T gg[4];
                    if constexpr (GD) {
                        TA ga[4];
                        ldg4(gsrc + pb + NZ * a + z4, ga);
#pragma unroll
                        for (int z = 0; z < 4; ++z) gg[z] = (T)ga[z];
                    } else {
                        ld4(gb + NZ * a + z4, gg);
                    }
#pragma unroll
                    for (int z = 0; z < 4; ++z) {
                        sg += gg[z] * fz[z4 + z];
                        sgd += gg[z] * dfz[z4 + z];
                    }
                }
                Dc += sgd * fa * fcc;
                Drj += sg * (dfa_half * fcc + fa * dfcj * fck);
                Drk += sg * (dfa_half * fcc + fa * fcj * dfck);
            }
            // dc/dx_j = (u_k - c u_j)/r_j ; dc/dx_k = (u_j - c u_k)/r_k
            const T gj0 = Drj * uj0 + Dc * (uk0 - cs_ * uj0) * ij;
            const T gj1 = Drj * uj1 + Dc * (uk1 - cs_ * uj1) * ij;
            const T gj2 = Drj * uj2 + Dc * (uk2 - cs_ * uj2) * ij;
            const T gk0 = Drk * uk0 + Dc * (uj0 - cs_ * uk0) * ik;
            const T gk1 = Drk * uk1 + Dc * (uj1 - cs_ * uk1) * ik;
            const T gk2 = Drk * uk2 + Dc * (uj2 - cs_ * uk2) * ik;
            T* o = pg + 6 * lane;
            o[0] = gj0; o[1] = gj1; o[2] = gj2;
            o[3] = gk0; o[4] = gk1; o[5] = gk2;
            fi0 += gj0 + gk0;
            fi1 += gj1 + gk1;
            fi2 += gj2 + gk2;
          }
          wave_sync();
          // diagonals of this batch: pair q = (d-1) n + a on diagonal d <= D,
          // q = full + a on the half diagonal d = n/2 of an even n
          const int d0 = P0 < full ? P0 / nang + 1 : half;
          const int d1 = P0 + nbat - 1 < full ? (P0 + nbat - 1) / nang + 1 : half;
          for (int u = lane; u < 3 * nang; u += 64) {
            const int t = u / 3, cc = u - 3 * t;
            T sum = T(0);
            for (int d = d0; d <= d1; ++d) {
              int qj, qk;   // the pairs (t, t+d) and (t-d, t)
              if (d <= D) {
                qj = (d - 1) * nang + t;
                const int a = t - d;
                qk = (d - 1) * nang + (a < 0 ? a + nang : a);
              } else {
                qj = t < half ? full + t : -1;
                qk = t >= half ? full + t - half : -1;
              }
              qj -= P0;
              qk -= P0;
              if (qj >= 0 && qj < nbat) sum += pg[6 * qj + cc];
              if (qk >= 0 && qk < nbat) sum += pg[6 * qk + 3 + cc];
            }
            const int jt = tag_of(nb + kNbStride * t) >> 8;
            Acc::add(&sF[3 * jt + cc], -sum);
          }
          wave_sync();
        }
        for (int off = 32; off > 0; off >>= 1) {
            fi0 += __shfl_xor(fi0, off);
            fi1 += __shfl_xor(fi1, off);
            fi2 += __shfl_xor(fi2, off);
        }
        if (lane == 0) {
            Acc::add(&sF[3 * il + 0], fi0);
            Acc::add(&sF[3 * il + 1], fi1);
            Acc::add(&sF[3 * il + 2], fi2);
        }
        wave_sync();
    }
    __syncthreads();
    for (int t = tid; t < 3 * n; t += blockDim.x) Acc::flush(sF[t], F, Fq, 3 * (size_t)a0 + t);
}

template <typename T>
static size_t forces_lds(int max_apm, int cap, int S, int nw, bool fixed = false, bool gd = false) {
    const int GL = kNR * S + kBlkPad * S * (S + 1) / 2;
    return ChunkStage<T>::bytes(max_apm, cap) +
           (fixed ? lds_bytes<unsigned long long>(3 * (size_t)max_apm) : lds_bytes<T>(3 * (size_t)max_apm)) +
           lds_bytes<T>((size_t)nw * cap * kNbStride) + lds_bytes<T>((size_t)nw * 64 * 6) +
           (gd ? 0 : lds_bytes<T>((size_t)nw * GL));
}

template <typename P>
hipError_t launch_forces(const Shape& sh, const AevConst<typename P::T>& c,
                         const int32_t* mol_off, const int32_t* species, const typename P::T* x,
                         Work<P>& w, typename P::T* F, hipStream_t st, const Timer& tm,
                         const EnergyArgs<P>& ea) {
    typedef typename P::T T;
    if (c.Dp > 2 * 16 * 64) return hipErrorInvalidValue;
    dim3 grid(sh.B, (sh.max_apm + sh.chunk - 1) / sh.chunk);
    int nw = kWaves;
    const bool fixed = sh.force_fixed != 0, gd = sh.force_path == 2;
    size_t lds = forces_lds<T>(sh.max_apm, sh.cap_nbr, sh.S, nw, fixed, gd);
    while (lds > kMaxLds && nw > 1) lds = forces_lds<T>(sh.max_apm, sh.cap_nbr, sh.S, nw /= 2, fixed, gd);
    if (lds > kMaxLds) return hipErrorInvalidValue;
    auto kern = gd ? (fixed ? (c.nZ == 4 ? k_forces<P, 4, true, true> : k_forces<P, 8, true, true>)
                            : (c.nZ == 4 ? k_forces<P, 4, false, true> : k_forces<P, 8, false, true>))
                   : (fixed ? (c.nZ == 4 ? k_forces<P, 4, true, false> : k_forces<P, 8, true, false>)
                            : (c.nZ == 4 ? k_forces<P, 4, false, false> : k_forces<P, 8, false, false>));
    hipError_t e = ensure_lds((const void*)kern, lds);
    if (e != hipSuccess) return e;
    tm.b("forces", st);
    hipLaunchKernelGGL(kern, grid, dim3(64 * nw), lds, st, c, sh.A, sh.max_apm, sh.chunk, sh.cap_nbr,
                       mol_off, species, x, w.nbr, w.nbr_cnt, w.row_of_atom, w.dG, F, w.Fq, ea);
    tm.e("forces", st);
    return hipGetLastError();
}

// ==========================================================================
// Second-order term of a Hessian-vector product.  With F = -sum_i (dG_i/dx)^T g_i
// (the force contraction above, g the dE/dAEV rows), the derivative of the
// energy gradient along v has two parts: the rows' own change (handled by
// running the force contraction on the rows' tangent) and the change of
// dG/dx itself with g held fixed.  This kernel forms the second part as the
// tangent of the force contraction along x + t v: every geometric quantity is
// carried as a (value, tangent) pair; the work split is k_forces'.
template <typename T> struct Du {
    T v, t;
};
template <typename T> __device__ inline Du<T> du(T v, T t = T(0)) { return Du<T>{v, t}; }
template <typename T> __device__ inline Du<T> operator+(Du<T> a, Du<T> b) { return {a.v + b.v, a.t + b.t}; }
template <typename T> __device__ inline Du<T> operator-(Du<T> a, Du<T> b) { return {a.v - b.v, a.t - b.t}; }
template <typename T> __device__ inline Du<T> operator-(Du<T> a) { return {-a.v, -a.t}; }
template <typename T> __device__ inline Du<T> operator*(Du<T> a, Du<T> b) { return {a.v * b.v, a.t * b.v + a.v * b.t}; }
template <typename T> __device__ inline Du<T> operator*(T s, Du<T> a) { return {s * a.v, s * a.t}; }
template <typename T> __device__ inline Du<T> operator+(Du<T> a, T s) { return {a.v + s, a.t}; }
template <typename T> __device__ inline Du<T> d_rcp(Du<T> a) {
    const T r = m_rcp(a.v);
    return {r, -a.t * r * r};
}
template <typename T> __device__ inline Du<T> d_sqrt(Du<T> a) {
    const T q = m_sqrt(a.v);
    return {q, T(0.5) * a.t * m_rcp(q)};
}
template <typename T> __device__ inline Du<T> d_exp(Du<T> a) {
    const T e = m_exp(a.v);
    return {e, e * a.t};
}
template <typename T> __device__ inline Du<T> d_powu(Du<T> a, T p) {
    if (!(a.v > T(0))) return {T(0), T(0)};
    const T y = m_powu(a.v, p);
    return {y, p * y * m_rcp(a.v) * a.t};
}
// fc(r) = cos(pi r / Rc)/2 + 1/2 and its derivative, both as pairs
template <typename T> __device__ inline void d_cutoff(Du<T> r, T pi_rc, Du<T>& fc, Du<T>& dfc) {
    const T cs = m_cos(pi_rc * r.v), sn = m_sin(pi_rc * r.v);
    fc = {T(0.5) * cs + T(0.5), -T(0.5) * pi_rc * sn * r.t};
    dfc = {-T(0.5) * pi_rc * sn, -T(0.5) * pi_rc * pi_rc * cs * r.t};
}

constexpr int kNbStrideT = 17;   // values dx dy dz r fc_r dfc_r fc_a dfc_a, then their tangents (odd stride: banks)

template <typename P, int NZ>
__global__ __launch_bounds__(256) void k_forces_tan(AevConst<typename P::T> c, int A, int max_apm,
                                                    int chunk, int cap,
                                                    const int32_t* __restrict__ mol_off,
                                                    const int32_t* __restrict__ species,
                                                    const typename P::T* __restrict__ x,
                                                    const typename P::T* __restrict__ vdir,
                                                    const uint16_t* __restrict__ nbr,
                                                    const int32_t* __restrict__ nbr_cnt,
                                                    const int32_t* __restrict__ row_of_atom,
                                                    const typename P::TA* __restrict__ dG,
                                                    typename P::T* __restrict__ Tout) {
    typedef typename P::T T;
    typedef typename P::TA TA;
    typedef Du<T> D;
    constexpr int NA = kNAZ / NZ;
    extern __shared__ __align__(16) char smem[];
    const int b = blockIdx.x;
    const int a0 = mol_off[b], n = mol_off[b + 1] - a0;
    if (n <= 0 || n > max_apm || a0 < 0 || a0 + n > A) return;
    const int i0 = blockIdx.y * chunk;
    if (i0 >= n) return;
    const int nc = min(chunk, n - i0);
    const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6, nw = blockDim.x >> 6;
    const int S = c.S, RL = kNR * S, NB = S * (S + 1) / 2;
    const int GL = RL + kBlkPad * NB;

    LdsBump lb(smem);
    ChunkStage<T> cs;
    cs.take(lb, max_apm, cap);
    T* sv = lb.take<T>(3 * (size_t)max_apm);   // the direction v of the molecule
    T* sF = lb.take<T>(3 * (size_t)max_apm);
    T* nb = lb.take<T>((size_t)nw * cap * kNbStrideT) + (size_t)wave * cap * kNbStrideT;
    int* nsp = lb.take<int>((size_t)nw * cap) + (size_t)wave * cap;
    int* nid = lb.take<int>((size_t)nw * cap) + (size_t)wave * cap;
    T* g = lb.take<T>((size_t)nw * GL) + (size_t)wave * GL;

    cs.load(x, species, S, a0, n, i0, nc, cap, nbr, nbr_cnt, row_of_atom);
    for (int t = tid; t < 3 * n; t += blockDim.x) {
        sv[t] = vdir[3 * (size_t)a0 + t];
        sF[t] = T(0);
    }
    __syncthreads();
    for (int ic = wave; ic < nc; ic += nw) {
        const int il = i0 + ic;
        const int cnt = cs.ccnt[ic];
        const int nang = cnt & 0xffff, nall = cnt >> 16;
        // the atom's dE/dAEV row, laid out as in k_forces
        {
            const TA* src = dG + (size_t)cs.crow[ic] * c.Dp;
            for (int e = lane; e < c.D; e += 64) {
                const int le = e < RL ? e : RL + kBlkPad * ((e - RL) / kNAZ) + (e - RL) % kNAZ;
                g[le] = (T)src[e];
            }
        }
        // neighbours with tangents: d_j = x_j - x_i moves along v_j - v_i
        {
            const T xi0 = cs.sx[3 * il], xi1 = cs.sx[3 * il + 1], xi2 = cs.sx[3 * il + 2];
            const T vi0 = sv[3 * il], vi1 = sv[3 * il + 1], vi2 = sv[3 * il + 2];
            for (int t = lane; t < nall; t += 64) {
                const int j = cs.clst[(size_t)ic * cap + t];
                const T d0 = cs.sx[3 * j] - xi0, d1 = cs.sx[3 * j + 1] - xi1, d2 = cs.sx[3 * j + 2] - xi2;
                const T t0 = sv[3 * j] - vi0, t1 = sv[3 * j + 1] - vi1, t2 = sv[3 * j + 2] - vi2;
                const D r = d_sqrt(D{d0 * d0 + d1 * d1 + d2 * d2, T(2) * (d0 * t0 + d1 * t1 + d2 * t2)});
                D fcr, dfcr, fca = du(T(0)), dfca = du(T(0));
                d_cutoff(r, c.pi_rcr, fcr, dfcr);
                if (t < nang) d_cutoff(r, c.pi_rca, fca, dfca);
                T* e = nb + kNbStrideT * t;
                e[0] = d0; e[1] = d1; e[2] = d2; e[3] = r.v; e[4] = fcr.v; e[5] = dfcr.v; e[6] = fca.v; e[7] = dfca.v;
                e[8] = t0; e[9] = t1; e[10] = t2; e[11] = r.t; e[12] = fcr.t; e[13] = dfcr.t; e[14] = fca.t; e[15] = dfca.t;
                nsp[t] = cs.ssp[j];
                nid[t] = j;
            }
        }
        wave_sync();
        T fi0 = 0, fi1 = 0, fi2 = 0;   // tangent force on the central atom, per lane
        // radial: lane per (neighbour, group of 4 shifts)
        for (int it = lane; it < ((4 * nall + 63) & ~63); it += 64) {
            const bool act = it < 4 * nall;
            const int t = act ? (it >> 2) : 0, q = it & 3;
            D dEdr = du(T(0));
            const T* e = nb + kNbStrideT * t;
            if (act) {
                const D r{e[3], e[11]}, fc{e[4], e[12]}, dfc{e[5], e[13]};
                const T* gg = g + kNR * nsp[t] + 4 * q;
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    const D d = r + (-c.shf_r[4 * q + kk]);
                    const D ex = c.radial_pref * d_exp(-c.eta_r * (d * d));
                    dEdr = dEdr + gg[kk] * (ex * ((T(-2) * c.eta_r) * (d * fc) + dfc));
                }
            }
            dEdr.v += __shfl_xor(dEdr.v, 1);
            dEdr.t += __shfl_xor(dEdr.t, 1);
            dEdr.v += __shfl_xor(dEdr.v, 2);
            dEdr.t += __shfl_xor(dEdr.t, 2);
            if (act && q == 0) {
                const D inv = d_rcp(D{e[3], e[11]});
                const D f0 = dEdr * (D{e[0], e[8]} * inv), f1 = dEdr * (D{e[1], e[9]} * inv),
                        f2 = dEdr * (D{e[2], e[10]} * inv);
                const int j = nid[t];
                lds_add(&sF[3 * j + 0], -f0.t);
                lds_add(&sF[3 * j + 1], -f1.t);
                lds_add(&sF[3 * j + 2], -f2.t);
                fi0 += f0.t;
                fi1 += f1.t;
                fi2 += f2.t;
            }
        }
        // angular: lane per neighbour pair
        const int npair = nang * (nang - 1) / 2;
        for (int p = lane; p < npair; p += 64) {
            int j, k;
            decode_pair_rot(p, nang, j, k);
            const T* ej = nb + kNbStrideT * j;
            const T* ek = nb + kNbStrideT * k;
            const D rj{ej[3], ej[11]}, rk{ek[3], ek[11]};
            const D ij = d_rcp(rj), ik = d_rcp(rk);
            const D uj0 = D{ej[0], ej[8]} * ij, uj1 = D{ej[1], ej[9]} * ij, uj2 = D{ej[2], ej[10]} * ij;
            const D uk0 = D{ek[0], ek[8]} * ik, uk1 = D{ek[1], ek[9]} * ik, uk2 = D{ek[2], ek[10]} * ik;
            D cs_ = uj0 * uk0 + uj1 * uk1 + uj2 * uk2;
            if (cs_.v > T(1)) cs_ = du(T(1));
            if (cs_.v < T(-1)) cs_ = du(T(-1));
            const D cp = c.angle_scale * cs_;
            const D sn = d_sqrt(D{T(1), T(0)} - cp * cp);
            const D fcj{ej[6], ej[14]}, fck{ek[6], ek[14]}, dfcj{ej[7], ej[15]}, dfck{ek[7], ek[15]};
            const D fcc = fcj * fck;
            const D rm = T(0.5) * (rj + rk);
            const T* gb = g + RL + kBlkPad * pair_index(nsp[j], nsp[k], S);
            D fz[NZ], dfz[NZ];
            const D isn = d_rcp(sn);
#pragma unroll
            for (int z = 0; z < NZ; ++z) {
                const D cz = c.cos_z[z] * cp + c.sin_z[z] * sn;
                const D hh = T(0.5) * (cz + T(1));
                const D hp = d_powu(hh, c.zeta - T(1));
                fz[z] = T(2) * (hp * hh);
                const D dcz = c.angle_scale * (du(c.cos_z[z]) - c.sin_z[z] * (cp * isn));
                dfz[z] = c.zeta * (hp * dcz);
            }
            D Dc = du(T(0)), Drj = du(T(0)), Drk = du(T(0));
#pragma unroll
            for (int a = 0; a < NA; ++a) {
                const D d = rm + (-c.shf_a[a]);
                const D fa = d_exp(-c.eta_a * (d * d));
                const D dfa_half = -c.eta_a * (d * fa);
                D sg = du(T(0)), sgd = du(T(0));
#pragma unroll
                for (int z = 0; z < NZ; ++z) {
                    const T gv = gb[NZ * a + z];
                    sg = sg + gv * fz[z];
                    sgd = sgd + gv * dfz[z];
                }
                Dc = Dc + sgd * (fa * fcc);
                Drj = Drj + sg * (dfa_half * fcc + fa * (dfcj * fck));
                Drk = Drk + sg * (dfa_half * fcc + fa * (fcj * dfck));
            }
            const D gj0 = Drj * uj0 + Dc * ((uk0 - cs_ * uj0) * ij);
            const D gj1 = Drj * uj1 + Dc * ((uk1 - cs_ * uj1) * ij);
            const D gj2 = Drj * uj2 + Dc * ((uk2 - cs_ * uj2) * ij);
            const D gk0 = Drk * uk0 + Dc * ((uj0 - cs_ * uk0) * ik);
            const D gk1 = Drk * uk1 + Dc * ((uj1 - cs_ * uk1) * ik);
            const D gk2 = Drk * uk2 + Dc * ((uj2 - cs_ * uk2) * ik);
            const int jj = nid[j], kk = nid[k];
            lds_add(&sF[3 * jj + 0], -gj0.t);
            lds_add(&sF[3 * jj + 1], -gj1.t);
            lds_add(&sF[3 * jj + 2], -gj2.t);
            lds_add(&sF[3 * kk + 0], -gk0.t);
            lds_add(&sF[3 * kk + 1], -gk1.t);
            lds_add(&sF[3 * kk + 2], -gk2.t);
            fi0 += gj0.t + gk0.t;
            fi1 += gj1.t + gk1.t;
            fi2 += gj2.t + gk2.t;
        }
        for (int off = 32; off > 0; off >>= 1) {
            fi0 += __shfl_xor(fi0, off);
            fi1 += __shfl_xor(fi1, off);
            fi2 += __shfl_xor(fi2, off);
        }
        if (lane == 0) {
            lds_add(&sF[3 * il + 0], fi0);
            lds_add(&sF[3 * il + 1], fi1);
            lds_add(&sF[3 * il + 2], fi2);
        }
        wave_sync();
    }
    __syncthreads();
    for (int t = tid; t < 3 * n; t += blockDim.x) {
        T val = sF[t];
        if (val != T(0)) gbl_add(&Tout[3 * (size_t)a0 + t], val);
    }
}

template <typename T>
static size_t forces_tan_lds(int max_apm, int cap, int S, int nw) {
    const int GL = kNR * S + kBlkPad * S * (S + 1) / 2;
    return ChunkStage<T>::bytes(max_apm, cap) + 2 * lds_bytes<T>(3 * (size_t)max_apm) +
           lds_bytes<T>((size_t)nw * cap * kNbStrideT) + 2 * lds_bytes<int>((size_t)nw * cap) +
           lds_bytes<T>((size_t)nw * GL);
}

template <typename P>
hipError_t launch_forces_tan(const Shape& sh, const AevConst<typename P::T>& c,
                             const int32_t* mol_off, const int32_t* species, const typename P::T* x,
                             const typename P::T* v, Work<P>& w, typename P::T* Tout, hipStream_t st,
                             const Timer& tm) {
    typedef typename P::T T;
    dim3 grid(sh.B, (sh.max_apm + sh.chunk - 1) / sh.chunk);
    int nw = kWaves;
    size_t lds = forces_tan_lds<T>(sh.max_apm, sh.cap_nbr, sh.S, nw);
    while (lds > kMaxLds && nw > 1) lds = forces_tan_lds<T>(sh.max_apm, sh.cap_nbr, sh.S, nw /= 2);
    if (lds > kMaxLds) return hipErrorInvalidValue;
    auto kern = c.nZ == 4 ? k_forces_tan<P, 4> : k_forces_tan<P, 8>;
    hipError_t e = ensure_lds((const void*)kern, lds);
    if (e != hipSuccess) return e;
    tm.b("forces_tan", st);
    hipLaunchKernelGGL(kern, grid, dim3(64 * nw), lds, st, c, sh.A, sh.max_apm, sh.chunk, sh.cap_nbr,
                       mol_off, species, x, v, w.nbr, w.nbr_cnt, w.row_of_atom, w.dG, Tout);
    tm.e("forces_tan", st);
    return hipGetLastError();
}

// y -= x over n values
template <typename T>
__global__ __launch_bounds__(256) void k_sub(size_t n, const T* __restrict__ xv, T* __restrict__ y) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] -= xv[i];
}
template <typename T> hipError_t launch_sub(size_t n, const T* xv, T* y, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sub<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, xv, y);
    return hipGetLastError();
}
template hipError_t launch_sub<float>(size_t, const float*, float*, hipStream_t);
template hipError_t launch_sub<double>(size_t, const double*, double*, hipStream_t);
template hipError_t launch_forces_tan<PrecF64>(const Shape&, const AevConst<double>&, const int32_t*,
                                               const int32_t*, const double*, const double*,
                                               Work<PrecF64>&, double*, hipStream_t, const Timer&);
template hipError_t launch_forces_tan<PrecF32>(const Shape&, const AevConst<float>&, const int32_t*,
                                               const int32_t*, const float*, const float*,
                                               Work<PrecF32>&, float*, hipStream_t, const Timer&);

// ==========================================================================
// energies: one wave per molecule, FP64 sum of the atomic energies in a fixed
// order.  e_atom = scale * ( mean_m (sum_t Epart + b4) ) + sae_scaled.
// With fixed-point force sums (Fq != null) the same wave also turns its
// molecule's integer force sums into F.  accumulate adds E (and F) to what
// the outputs hold.
template <typename P>
__global__ __launch_bounds__(256) void k_energy(int A, int B, int M, int NT, double scale,
                                                const int32_t* __restrict__ mol_off,
                                                const int32_t* __restrict__ species, int S,
                                                const int32_t* __restrict__ row_of_atom,
                                                const typename P::TA* __restrict__ Epart,
                                                const typename P::TA* __restrict__ b4,
                                                const double* __restrict__ sae,
                                                double* __restrict__ E,
                                                const unsigned long long* __restrict__ Fq,
                                                typename P::T* __restrict__ F, int accumulate,
                                                const int32_t* __restrict__ dcnt) {
    typedef typename P::T T;
    const int b = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = lane_id();
    if (b >= B || (dcnt && b >= dcnt[0])) return;   // past the batch (or its padding)
    int a0 = mol_off[b], a1 = mol_off[b + 1];
    if (a0 < 0 || a1 < a0 || a1 > A) a1 = a0 = 0;
    if (Fq)
        for (int t = 3 * a0 + lane; t < 3 * a1; t += 64) {
            const T f = (T)((double)(long long)Fq[t] * (1.0 / kForceFix));
            F[t] = accumulate ? F[t] + f : f;
        }
    const double v = molecule_energy<P>(a0, a1, M, NT, scale, species, S, row_of_atom, Epart, b4, sae);
    if (lane == 0) E[b] = accumulate ? E[b] + v : v;
}

template <typename P>
EnergyArgs<P> energy_args(const Shape& sh, const DevWeights<P>& wt, Work<P>& w, double* E, bool accumulate) {
    EnergyArgs<P> ea;
    ea.E = E;
    ea.Epart = w.Epart;
    ea.b4 = wt.b4;
    ea.sae = wt.sae;
    ea.scale = sh.energy_scale;
    ea.M = sh.M;
    ea.NT = w.epart_nt;
    ea.B = sh.B;
    ea.accumulate = accumulate ? 1 : 0;
    ea.dcnt = sh.dev_counts ? w.dcnt : nullptr;
    return ea;
}

template <typename P>
hipError_t launch_energy(const Shape& sh, const DevWeights<P>& wt, const int32_t* mol_off,
                         const int32_t* species, Work<P>& w, double* E, typename P::T* F,
                         bool accumulate, hipStream_t st, const Timer& tm) {
    tm.b("energy", st);
    hipLaunchKernelGGL(k_energy<P>, dim3((sh.B + 3) / 4), dim3(256), 0, st, sh.A, sh.B, sh.M,
                       w.epart_nt, sh.energy_scale, mol_off, species, sh.S, w.row_of_atom,
                       w.Epart, wt.b4, wt.sae, E, (sh.force_fixed && F) ? w.Fq : nullptr, F,
                       accumulate ? 1 : 0, sh.dev_counts ? w.dcnt : nullptr);
    tm.e("energy", st);
    return hipGetLastError();
}

#define NNP_INST(P)                                                                            \
    template hipError_t launch_prep<P>(const Shape&, const int32_t*, const int32_t*, Work<P>&,  \
                                       hipStream_t, const Timer&);                             \
    template hipError_t launch_neighbours<P>(const Shape&, const AevConst<P::T>&,              \
                                             const int32_t*, const int32_t*, const P::T*,      \
                                             P::T*, bool, Work<P>&, hipStream_t, const Timer&); \
    template hipError_t launch_aev<P>(const Shape&, const AevConst<P::T>&, const int32_t*,     \
                                      const int32_t*, const P::T*, Work<P>&, P::T*,            \
                                      hipStream_t, const Timer&, const NbrFuse<P::T>&);        \
    template hipError_t launch_prep_features<P>(const Shape&, const AevConst<P::T>&,           \
                                                const int32_t*, const int32_t*, const P::T*,     \
                                                P::T*, bool, Work<P>&, P::T*, hipStream_t,       \
                                                const Timer&);                                   \
    template hipError_t launch_features<P>(const Shape&, const AevConst<P::T>&,                \
                                           const int32_t*, const int32_t*, const P::T*, P::T*, \
                                           bool, Work<P>&, P::T*, hipStream_t, const Timer&);  \
    template hipError_t launch_forces<P>(const Shape&, const AevConst<P::T>&, const int32_t*,  \
                                         const int32_t*, const P::T*, Work<P>&, P::T*,         \
                                         hipStream_t, const Timer&, const EnergyArgs<P>&);     \
    template EnergyArgs<P> energy_args<P>(const Shape&, const DevWeights<P>&, Work<P>&,        \
                                          double*, bool);                                      \
    template hipError_t launch_aev_jvp<P>(const Shape&, const AevConst<P::T>&, const int32_t*, \
                                          const int32_t*, const P::T*, const P::T*, Work<P>&,  \
                                          P::TS*, hipStream_t, const Timer&);                  \
    template hipError_t launch_energy<P>(const Shape&, const DevWeights<P>&, const int32_t*,   \
                                         const int32_t*, Work<P>&, double*, P::T*, bool,       \
                                         hipStream_t, const Timer&);

NNP_INST(PrecF64)
NNP_INST(PrecF32)
NNP_INST(PrecBF16)

}  // namespace nnp
