// nnp_runtime.cpp -- host side of the C ABI declared in include/nnp.h.
//
// Owns validation, weight packing for the chosen precision, the workspace
// sized for the declared capacity (the only device allocations), the launch
// sequence of one evaluation, per-kernel event timing and error reporting.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "nnp.h"
#include "nnp_internal.h"

using namespace nnp;

namespace {

thread_local std::string g_err;

nnp_status fail(nnp_status code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t _e = (expr);                                                         \
        if (_e != hipSuccess)                                                           \
            return fail(_e == hipErrorOutOfMemory ? NNP_E_NOMEM : NNP_E_DEVICE,         \
                        std::string(#expr) + ": " + hipGetErrorString(_e));             \
    } while (0)

struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

int pad_to(int v, int q) { return ((v + q - 1) / q) * q; }

struct EventPair {
    const char* name;
    hipEvent_t a, b;
};

// one captured evaluation, valid for exactly these shapes, pointers and stream
struct GraphEntry {
    int A = 0, B = 0;
    uint32_t flags = 0;
    const void* ptr[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    hipStream_t stream = nullptr;
    hipGraphExec_t exec = nullptr;
    bool same(int a, int b, uint32_t f, const void* const* p, hipStream_t s) const {
        if (a != A || b != B || f != flags || s != stream) return false;
        for (int i = 0; i < 6; ++i)
            if (p[i] != ptr[i]) return false;
        return true;
    }
};
constexpr size_t kMaxGraphs = 8;

}  // namespace

// ---------------------------------------------------------------------------
struct nnp_handle {
    // model
    int S = 0, nR = 0, nA = 0, nZ = 0, D = 0, M = 0, L = 0;
    std::vector<int> widths;
    int precision = 0, device = 0;
    int max_atoms = 0, max_mols = 0, max_apm = 0;
    double energy_scale = 1.0, celu_alpha = 0.1;
    std::vector<double> sae;
    AevConst<float> cf{};
    AevConst<double> cd{};
    Shape shape{};
    int64_t n_params = 0;
    // element networks of their own widths: packed index -> index in the
    // zero-padded uniform layout (host and device copies); gradients are
    // formed in that layout (gpad) and gathered
    bool het = false;
    int64_t n_int = 0;
    std::vector<int32_t> pmap;
    int32_t* dmap = nullptr;
    void* gpad = nullptr;

    // device memory
    std::vector<void*> allocs;
    DevWeights<PrecF64> w64{};
    DevWeights<PrecF32> w32{};
    DevWeights<PrecBF16> w16{};
    Work<PrecF64> k64{};
    Work<PrecF32> k32{};
    Work<PrecBF16> k16{};
    // the second part of a pipelined evaluation: its own row buffers (the
    // per-atom arrays are shared, indexed by absolute atom number), a second
    // stream (default priority) and the events that order the two parts
    bool pipe_ready = false;
    Work<PrecF64> k64b{};
    Work<PrecF32> k32b{};
    Work<PrecBF16> k16b{};
    hipStream_t st2 = nullptr;
    hipEvent_t pev[4] = {nullptr, nullptr, nullptr, nullptr};
    int32_t* flag = nullptr;
    int8_t* zlut = nullptr;       // device [kZLut]: element of each atomic number, or null
    hipStream_t last_stream = nullptr;

    // training backward workspace (allocated on its first call)
    bool train_ready = false;
    TrainWork<PrecF64> t64{};
    TrainWork<PrecF32> t32{};
    void* train_F = nullptr;      // [max_atoms][3] coordinate type
    double* train_E = nullptr;    // [max_mols]
    NetLayout nl{};

    // captured evaluations (most recent last), and how often graphs were
    // captured and replayed
    std::vector<GraphEntry> graphs;
    int64_t n_captures = 0, n_replays = 0;

    // tunable knobs as set by the caller (0 = automatic)
    int32_t knob[NNP_N_KNOBS] = {};

    // timing
    bool timing = false;
    std::string timing_only;           // time only launches of this name (empty: all)
    std::vector<EventPair> pending;
    std::vector<hipEvent_t> free_events;
    std::map<std::string, std::pair<int64_t, double>> totals;

    void* dalloc(size_t bytes, hipError_t& e) {
        void* p = nullptr;
        e = hipMalloc(&p, bytes ? bytes : 16);
        if (e == hipSuccess) allocs.push_back(p);
        return p;
    }
    hipEvent_t ev() {
        if (!free_events.empty()) {
            hipEvent_t e = free_events.back();
            free_events.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        (void)hipEventCreate(&e);
        return e;
    }
};

namespace {

void tm_begin(void* ctx, const char* name, hipStream_t s) {
    nnp_handle* h = (nnp_handle*)ctx;
    if (!h->timing_only.empty() && h->timing_only != name) return;
    EventPair p{name, h->ev(), h->ev()};
    (void)hipEventRecord(p.a, s);
    h->pending.push_back(p);
}
void tm_end(void* ctx, const char* name, hipStream_t s) {
    nnp_handle* h = (nnp_handle*)ctx;
    if (!h->timing_only.empty() && h->timing_only != name) return;
    for (auto it = h->pending.rbegin(); it != h->pending.rend(); ++it)
        if (it->name == name) {
            (void)hipEventRecord(it->b, s);
            return;
        }
}
Timer make_timer(nnp_handle* h) {
    Timer t{};
    if (h->timing) {
        t.begin = tm_begin;
        t.end = tm_end;
        t.ctx = h;
    }
    return t;
}

template <typename T> void fill_const(AevConst<T>& c, const nnp_model_params* p, int D, int Dp) {
    c.S = p->n_species;
    c.nR = p->n_shf_r;
    c.nA = p->n_shf_a;
    c.nZ = p->n_shf_z;
    c.D = D;
    c.Dp = Dp;
    c.rcr = (T)p->rcr;
    c.rca = (T)p->rca;
    c.rcr2 = (T)(p->rcr * p->rcr);
    c.rca2 = (T)(p->rca * p->rca);
    c.eta_r = (T)p->eta_r;
    c.eta_a = (T)p->eta_a;
    c.zeta = (T)p->zeta;
    c.angle_scale = (T)p->angle_scale;
    c.radial_pref = (T)p->radial_pref;
    c.pi_rcr = (T)(M_PI / p->rcr);
    c.pi_rca = (T)(M_PI / p->rca);
    for (int k = 0; k < p->n_shf_r; ++k) c.shf_r[k] = (T)p->shf_r[k];
    for (int a = 0; a < p->n_shf_a; ++a) c.shf_a[a] = (T)p->shf_a[a];
    for (int z = 0; z < p->n_shf_z; ++z) {
        c.cos_z[z] = (T)std::cos(p->shf_z[z]);
        c.sin_z[z] = (T)std::sin(p->shf_z[z]);
    }
}

template <typename TS> TS to_store(double v);
template <> float to_store<float>(double v) { return (float)v; }
template <> double to_store<double>(double v) { return v; }
template <> bf16_t to_store<bf16_t>(double v) { return f2bf((float)v); }

// Pack FP64 master weights [m][s][layer]{W, b} into the device layouts.
template <typename P> nnp_status upload_weights(nnp_handle* h, DevWeights<P>& dw,
                                                const double* w, bool allocate) {
    typedef typename P::TS TS;
    typedef typename P::TA TA;
    std::vector<double> padded;
    if (h->het) {   // into the zero-padded uniform layout
        padded.assign((size_t)h->n_int, 0.0);
        for (size_t i = 0; i < h->pmap.size(); ++i) padded[h->pmap[i]] = w[i];
        w = padded.data();
    }
    const Shape& sh = h->shape;
    const int S = h->S, M = h->M, D = h->D, Dp = sh.Dp;
    const int o1 = h->widths[1], o2 = h->widths[2], o3 = h->widths[3];
    const int H1 = sh.H1, H2 = sh.H2, H3 = sh.H3;
    std::vector<TS> W1((size_t)S * M * H1 * Dp, to_store<TS>(0.0)), W1T(W1.size(), to_store<TS>(0.0));
    std::vector<TS> W2((size_t)S * M * H2 * H1, to_store<TS>(0.0)), W2T(W2.size(), to_store<TS>(0.0));
    std::vector<TS> W3((size_t)S * M * H3 * H2, to_store<TS>(0.0)), W3T(W3.size(), to_store<TS>(0.0));
    std::vector<TA> b1((size_t)S * M * H1, 0), b2((size_t)S * M * H2, 0), b3((size_t)S * M * H3, 0);
    std::vector<TA> w4((size_t)S * M * H3, 0), b4((size_t)S * M, 0);
    std::vector<double> sae(S, 0.0);   // summed in FP64: self-energies dwarf the network part
    const size_t net = (size_t)o1 * D + o1 + (size_t)o2 * o1 + o2 + (size_t)o3 * o2 + o3 + o3 + 1;
    for (int m = 0; m < M; ++m)
        for (int s = 0; s < S; ++s) {
            const double* p = w + ((size_t)m * S + s) * net;
            for (int n = 0; n < o1; ++n)
                for (int k = 0; k < D; ++k) {
                    TS v = to_store<TS>(p[(size_t)n * D + k]);
                    W1[((size_t)s * M * H1 + (size_t)m * H1 + n) * Dp + k] = v;
                    W1T[((size_t)s * Dp + k) * M * H1 + (size_t)m * H1 + n] = v;
                }
            p += (size_t)o1 * D;
            for (int n = 0; n < o1; ++n) b1[(size_t)s * M * H1 + (size_t)m * H1 + n] = (TA)p[n];
            p += o1;
            const size_t sm = (size_t)s * M + m;
            for (int n = 0; n < o2; ++n)
                for (int k = 0; k < o1; ++k) {
                    TS v = to_store<TS>(p[(size_t)n * o1 + k]);
                    W2[(sm * H2 + n) * H1 + k] = v;
                    W2T[(sm * H1 + k) * H2 + n] = v;
                }
            p += (size_t)o2 * o1;
            for (int n = 0; n < o2; ++n) b2[sm * H2 + n] = (TA)p[n];
            p += o2;
            for (int n = 0; n < o3; ++n)
                for (int k = 0; k < o2; ++k) {
                    TS v = to_store<TS>(p[(size_t)n * o2 + k]);
                    W3[(sm * H3 + n) * H2 + k] = v;
                    W3T[(sm * H2 + k) * H3 + n] = v;
                }
            p += (size_t)o3 * o2;
            for (int n = 0; n < o3; ++n) b3[sm * H3 + n] = (TA)p[n];
            p += o3;
            for (int n = 0; n < o3; ++n) w4[sm * H3 + n] = (TA)p[n];
            p += o3;
            b4[sm] = (TA)p[0];
        }
    for (int s = 0; s < S; ++s) sae[s] = h->energy_scale * (h->sae.empty() ? 0.0 : h->sae[s]);
    // fragment-order copies of the per-model matrices (the fused kernel's
    // weight operands), one [N][K] matrix per element and model
    auto fragments = [&](const std::vector<TS>& src, int N, int K) {
        std::vector<TS> dst(src.size());
        for (size_t sm = 0; sm < (size_t)S * M; ++sm)
            for (int n = 0; n < N; ++n)
                for (int k = 0; k < K; ++k)
                    dst[sm * N * K + frag_index<TS>(n, k, K)] = src[(sm * N + n) * K + k];
        return dst;
    };
    const std::vector<TS> W2f = fragments(W2, H2, H1), W3f = fragments(W3, H3, H2);
    const std::vector<TS> W3Tf = fragments(W3T, H2, H3), W2Tf = fragments(W2T, H1, H2);
    // the layer-1 weights in fragment order for the register-operand GEMMs
    // (BF16): one [M*H1][Dp] matrix and its transpose per element
    std::vector<TS> W1f, W1Tf;
    if (std::is_same<TS, bf16_t>::value) {
        const int N1 = M * H1;
        W1f.resize(W1.size());
        W1Tf.resize(W1T.size());
        for (size_t e = 0; e < (size_t)S; ++e)
            for (int n = 0; n < N1; ++n)
                for (int k = 0; k < Dp; ++k) {
                    W1f[e * N1 * Dp + frag_index<TS>(n, k, Dp)] = W1[(e * N1 + n) * Dp + k];
                    W1Tf[e * N1 * Dp + frag_index<TS>(k, n, N1)] = W1[(e * N1 + n) * Dp + k];
                }
    }
    hipError_t e = hipSuccess;
    auto put = [&](auto*& dst, const auto& src) -> bool {
        size_t bytes = src.size() * sizeof(src[0]);
        if (allocate) {
            dst = (std::remove_reference_t<decltype(dst)>)h->dalloc(bytes, e);
            if (e != hipSuccess) return false;
        }
        e = hipMemcpy(dst, src.data(), bytes, hipMemcpyHostToDevice);
        return e == hipSuccess;
    };
    if (!put(dw.W1, W1) || !put(dw.W1T, W1T) || !put(dw.b1, b1) || !put(dw.W2, W2) ||
        !put(dw.W2T, W2T) || !put(dw.b2, b2) || !put(dw.W3, W3) || !put(dw.W3T, W3T) ||
        !put(dw.b3, b3) || !put(dw.w4, w4) || !put(dw.b4, b4) || !put(dw.sae, sae) ||
        !put(dw.W2f, W2f) || !put(dw.W3f, W3f) || !put(dw.W3Tf, W3Tf) || !put(dw.W2Tf, W2Tf) ||
        (!W1f.empty() && (!put(dw.W1f, W1f) || !put(dw.W1Tf, W1Tf))))
        return fail(e == hipErrorOutOfMemory ? NNP_E_NOMEM : NNP_E_DEVICE,
                    std::string("weight upload: ") + hipGetErrorString(e));
    return NNP_OK;
}

// Row buffers of the pipeline's second part (sized for the whole capacity:
// one part may hold nearly every atom); the per-atom arrays are the first
// workspace's.
template <typename P> nnp_status alloc_work2(nnp_handle* h, const Work<P>& w1, Work<P>& w) {
    typedef typename P::TS TS;
    typedef typename P::TA TA;
    const Shape& sh = h->shape;
    const size_t A = (size_t)std::max(h->max_atoms, 1), R = sh.Rcap;
    const int M = sh.M;
    hipError_t e = hipSuccess;
    w = w1;
#define ALLOC(field, bytes)                                                              \
    do {                                                                                 \
        w.field = (decltype(w.field))h->dalloc(bytes, e);                                \
        if (e != hipSuccess)                                                             \
            return fail(e == hipErrorOutOfMemory ? NNP_E_NOMEM : NNP_E_DEVICE,           \
                        std::string("pipeline workspace ") + #field + ": " + hipGetErrorString(e)); \
    } while (0)
    ALLOC(atom_of_row, sizeof(int32_t) * R);
    ALLOC(tile_species, sizeof(int32_t) * (R / sh.row_tile));
    ALLOC(info, sizeof(BucketInfo));
    const size_t nblk = (std::max(A, (size_t)h->max_mols) + kPrepBlock - 1) / kPrepBlock + 1;
    ALLOC(blk, sizeof(int32_t) * kMaxSpecies * nblk);
    ALLOC(G, sizeof(TS) * R * sh.Dp);
    ALLOC(H1, sizeof(TS) * R * M * sh.H1);
    ALLOC(H2, sizeof(TS) * R * M * sh.H2);
    ALLOC(DZ3, sizeof(TS) * R * M * sh.H3);
    ALLOC(DZ2, sizeof(TS) * R * M * sh.H2);
    ALLOC(DZ1, sizeof(TS) * R * M * sh.H1);
    ALLOC(Epart, sizeof(TA) * R * M * (sh.H3 / 64));
    ALLOC(dG, sizeof(typename P::TG) * R * sh.Dp);
#undef ALLOC
    HIP_TRY(hipMemset(w.info, 0, sizeof(BucketInfo)));
    HIP_TRY(hipMemset(w.G, 0, sizeof(TS) * R * sh.Dp));
    return NNP_OK;
}

template <typename P> nnp_status alloc_work(nnp_handle* h, Work<P>& w) {
    typedef typename P::TS TS;
    typedef typename P::TA TA;
    const Shape& sh = h->shape;
    const size_t A = (size_t)std::max(h->max_atoms, 1), R = sh.Rcap;
    const int M = sh.M;
    hipError_t e = hipSuccess;
#define ALLOC(field, bytes)                                                              \
    do {                                                                                 \
        w.field = (decltype(w.field))h->dalloc(bytes, e);                                \
        if (e != hipSuccess)                                                             \
            return fail(e == hipErrorOutOfMemory ? NNP_E_NOMEM : NNP_E_DEVICE,           \
                        std::string("workspace ") + #field + ": " + hipGetErrorString(e)); \
    } while (0)
    ALLOC(row_of_atom, sizeof(int32_t) * A);
    ALLOC(atom_of_row, sizeof(int32_t) * R);
    ALLOC(mol_of_atom, sizeof(int32_t) * A);
    ALLOC(tile_species, sizeof(int32_t) * (R / sh.row_tile));
    ALLOC(info, sizeof(BucketInfo));
    const size_t nblk = (std::max(A, (size_t)h->max_mols) + kPrepBlock - 1) / kPrepBlock + 1;
    ALLOC(blk, sizeof(int32_t) * kMaxSpecies * nblk);
    ALLOC(nbr, sizeof(uint16_t) * A * sh.cap_nbr);
    ALLOC(nbr_cnt, sizeof(int32_t) * A);
    ALLOC(G, sizeof(TS) * R * sh.Dp);
    ALLOC(H1, sizeof(TS) * R * M * sh.H1);
    ALLOC(H2, sizeof(TS) * R * M * sh.H2);
    ALLOC(DZ3, sizeof(TS) * R * M * sh.H3);
    ALLOC(DZ2, sizeof(TS) * R * M * sh.H2);
    ALLOC(DZ1, sizeof(TS) * R * M * sh.H1);
    ALLOC(Epart, sizeof(TA) * R * M * (sh.H3 / 64));
    ALLOC(dG, sizeof(typename P::TG) * R * sh.Dp);
    ALLOC(Fq, sizeof(unsigned long long) * 3 * A);
    ALLOC(moff, sizeof(int32_t) * ((size_t)h->max_mols + 1));
    ALLOC(dcnt, sizeof(int32_t) * 2);
    if (h->zlut) ALLOC(sp, sizeof(int32_t) * A);
#undef ALLOC
    w.epart_nt = sh.H3 / 64;
    w.flag = h->flag;
    w.zlut = h->zlut;
    // every row index the kernels may read must be in range from the start
    HIP_TRY(hipMemset(w.row_of_atom, 0, sizeof(int32_t) * A));
    HIP_TRY(hipMemset(w.nbr_cnt, 0, sizeof(int32_t) * A));
    HIP_TRY(hipMemset(w.info, 0, sizeof(BucketInfo)));
    // padding rows of the AEV operand are never written by the featuriser
    HIP_TRY(hipMemset(w.G, 0, sizeof(TS) * R * sh.Dp));
    return NNP_OK;
}

nnp_status check_batch(const nnp_handle* h, const nnp_batch* b) {
    if (!h || !b) return fail(NNP_E_INVALID, "null handle or batch");
    if (b->n_mols < 1) return fail(NNP_E_INVALID, "n_mols must be >= 1");
    if (b->n_mols > h->max_mols) return fail(NNP_E_CAPACITY, "n_mols exceeds max_mols");
    if (b->n_atoms < 0) return fail(NNP_E_INVALID, "n_atoms must be >= 0");
    if (b->n_atoms > h->max_atoms) return fail(NNP_E_CAPACITY, "n_atoms exceeds max_atoms");
    if (!b->mol_offsets) return fail(NNP_E_INVALID, "null mol_offsets");
    if (b->n_atoms > 0 && !b->species) return fail(NNP_E_INVALID, "null species");
    if (b->flags & ~(NNP_FLAG_GRAPH | NNP_FLAG_ACCUMULATE | NNP_FLAG_DEVICE_COUNTS))
        return fail(NNP_E_INVALID, "unknown flags");
    if ((b->flags & NNP_FLAG_DEVICE_COUNTS) && !b->counts)
        return fail(NNP_E_INVALID, "NNP_FLAG_DEVICE_COUNTS needs the device counts");
    if ((b->flags & NNP_FLAG_GRAPH) && !b->stream)
        return fail(NNP_E_INVALID, "graph replay needs a non-null stream");
    return NNP_OK;
}

template <typename P> Work<P>& work_of(nnp_handle* h);
template <> Work<PrecF64>& work_of<PrecF64>(nnp_handle* h) { return h->k64; }
template <> Work<PrecF32>& work_of<PrecF32>(nnp_handle* h) { return h->k32; }
template <> Work<PrecBF16>& work_of<PrecBF16>(nnp_handle* h) { return h->k16; }
template <typename P> Work<P>& work2_of(nnp_handle* h);
template <> Work<PrecF64>& work2_of<PrecF64>(nnp_handle* h) { return h->k64b; }
template <> Work<PrecF32>& work2_of<PrecF32>(nnp_handle* h) { return h->k32b; }
template <> Work<PrecBF16>& work2_of<PrecBF16>(nnp_handle* h) { return h->k16b; }
template <typename P> DevWeights<P>& weights_of(nnp_handle* h);
template <> DevWeights<PrecF64>& weights_of<PrecF64>(nnp_handle* h) { return h->w64; }
template <> DevWeights<PrecF32>& weights_of<PrecF32>(nnp_handle* h) { return h->w32; }
template <> DevWeights<PrecBF16>& weights_of<PrecBF16>(nnp_handle* h) { return h->w16; }
template <typename P> TrainWork<P>& train_of(nnp_handle* h);
template <> TrainWork<PrecF64>& train_of<PrecF64>(nnp_handle* h) { return h->t64; }
template <> TrainWork<PrecF32>& train_of<PrecF32>(nnp_handle* h) { return h->t32; }
template <typename T> const AevConst<T>& const_of(nnp_handle* h);
template <> const AevConst<float>& const_of<float>(nnp_handle* h) { return h->cf; }
template <> const AevConst<double>& const_of<double>(nnp_handle* h) { return h->cd; }

// the register-operand layer-1 GEMMs: BF16, 128-row buckets, both GEMMs'
// N (M*H1 forward, the padded AEV length backward) in 256-column tiles
bool l1_regs_supported(const nnp_handle* h) {
    const Shape& sh = h->shape;
    return h->precision == NNP_PREC_BF16_MLP && sh.row_tile == 128 && (sh.M * sh.H1) % 256 == 0 &&
           sh.Dp % 256 == 0;
}

// value in effect of a knob (automatic choices resolved)
int32_t knob_value(const nnp_handle* h, int k) {
    const Shape& sh = h->shape;
    const int32_t v = h->knob[k];
    switch (k) {
    case NNP_KNOB_MLP_PATH:
        if (v) return v;
        return mlp_fused_supported(sh.H1, sh.H2, sh.H3) ? 1 : 2;
    case NNP_KNOB_GEMM_STAGES: return v ? v : 2;
    case NNP_KNOB_CELL_MIN: return v ? v : 128;
    case NNP_KNOB_TAIL_TILE: return v ? v : 1;
    case NNP_KNOB_GEMM_WAVES: return v ? v : 8;
    case NNP_KNOB_ATOM_CHUNK:
        if (v) return v;
        return (int64_t)h->max_mols * ((h->max_apm + 15) / 16) >= 1024 ? 16 : 4;
    case NNP_KNOB_L1_PATH:
        if (v) return v;
        return l1_regs_supported(h) ? 2 : 1;
    case NNP_KNOB_FORCE_SUM: return v ? v : 1;
    case NNP_KNOB_FORCE_PATH: return v ? v : 2;
    case NNP_KNOB_PIPELINE: return v ? v : 1;
    }
    return 0;
}

// copy the resolved knobs into the handle's shape and drop captured graphs
void apply_knobs(nnp_handle* h) {
    h->shape.mlp_fused = knob_value(h, NNP_KNOB_MLP_PATH) == 1;
    h->shape.gemm_stages = knob_value(h, NNP_KNOB_GEMM_STAGES);
    h->shape.cell_min = knob_value(h, NNP_KNOB_CELL_MIN);
    h->shape.tail_tile = knob_value(h, NNP_KNOB_TAIL_TILE);
    h->shape.gemm_waves = knob_value(h, NNP_KNOB_GEMM_WAVES);
    h->shape.chunk = knob_value(h, NNP_KNOB_ATOM_CHUNK);
    h->shape.l1_path = knob_value(h, NNP_KNOB_L1_PATH);
    h->shape.force_fixed = knob_value(h, NNP_KNOB_FORCE_SUM) == 2;
    h->shape.force_path = knob_value(h, NNP_KNOB_FORCE_PATH);
    h->shape.pipeline = knob_value(h, NNP_KNOB_PIPELINE);
    for (auto& g : h->graphs) (void)hipGraphExecDestroy(g.exec);
    h->graphs.clear();
}

// element indices of the batch's atoms as the kernels after bucketing read
// them: the batch's own array, or the indices the bucketing kernels mapped
// from atomic numbers
template <typename P> const int32_t* elements_of(const Work<P>& w, const nnp_batch* b) {
    return w.zlut ? w.sp : b->species;
}

// launch bounds of a batch with device-side counts: the host's upper bounds
// rounded up to powers of two (at most the capacity), so batches of many
// sizes share one captured graph
int pow2_bound(int v, int cap) {
    int p = 1;
    while (p < v && p < cap) p <<= 1;
    return std::min(p, cap);
}
void launch_bounds(const nnp_handle* h, const nnp_batch* b, int& A, int& B) {
    A = b->n_atoms;
    B = b->n_mols;
    if (b->flags & NNP_FLAG_DEVICE_COUNTS) {
        A = pow2_bound(std::max(A, 1), h->max_atoms);
        B = pow2_bound(std::max(B, 1), h->max_mols);
    }
}

// The three stages of an evaluation of molecules [moff[0], moff[B]):
// featurisation (bucketing, neighbour lists, AEV rows), the networks, and
// the forces and energies.
template <typename P>
nnp_status stage_features(nnp_handle* h, const Shape& sh, const int32_t* moff, const int32_t* species,
                          const typename P::T* x, typename P::T* F, bool acc, Work<P>& w, hipStream_t st,
                          const Timer& tm) {
    const AevConst<typename P::T>& c = const_of<typename P::T>(h);
    HIP_TRY(launch_prep_features<P>(sh, c, moff, species, x, F, acc, w, nullptr, st, tm));
    return NNP_OK;
}
template <typename P>
nnp_status stage_finish(nnp_handle* h, const Shape& sh, const int32_t* moff, const int32_t* species,
                        const typename P::T* x, double* E, typename P::T* F, bool acc, Work<P>& w,
                        hipStream_t st, const Timer& tm) {
    const AevConst<typename P::T>& c = const_of<typename P::T>(h);
    const int32_t* sp = w.zlut ? w.sp : species;
    // with floating-point force sums the force kernel also sums the energies
    // (one launch fewer); fixed-point sums need the energy kernel after every
    // force workgroup, to convert them
    const bool fuse_e = F && sh.A > 0 && !sh.force_fixed;
    if (F && sh.A > 0)
        HIP_TRY(launch_forces<P>(sh, c, moff, sp, x, w, F, st, tm,
                                 fuse_e ? energy_args<P>(sh, weights_of<P>(h), w, E, acc) : EnergyArgs<P>()));
    if (!fuse_e)
        HIP_TRY(launch_energy<P>(sh, weights_of<P>(h), moff, sp, w, E, sh.A > 0 ? F : nullptr, acc, st, tm));
    return NNP_OK;
}

// Pipelined evaluation in two parts (molecules [0, B/2) and [B/2, B)) on two
// streams: the second part's featurisation (vector ALU work) runs while the
// first part's networks (matrix-core work) run, and the first part's forces
// while the second part's networks run; the two network stages run one after
// the other, so no two instances of a kernel run together.
// The pipeline's second workspace, stream and events, made when the knob
// first selects the pipelined evaluation (at creation when it is the
// automatic choice).
nnp_status ensure_pipeline(nnp_handle* h) {
    if (h->shape.pipeline != 2 || h->pipe_ready) return NNP_OK;
    DeviceGuard dg(h->device);
    if (!dg.ok) return fail(NNP_E_DEVICE, "hipSetDevice failed");
    nnp_status rc;
    if (h->precision == NNP_PREC_FP64) rc = alloc_work2<PrecF64>(h, h->k64, h->k64b);
    else if (h->precision == NNP_PREC_FP32) rc = alloc_work2<PrecF32>(h, h->k32, h->k32b);
    else rc = alloc_work2<PrecBF16>(h, h->k16, h->k16b);
    if (rc) return rc;
    if (!h->st2) HIP_TRY(hipStreamCreateWithFlags(&h->st2, hipStreamNonBlocking));
    for (auto& e : h->pev)
        if (!e) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    h->pipe_ready = true;
    return NNP_OK;
}

template <typename P>
nnp_status run_forward_split(nnp_handle* h, const nnp_batch* b, const typename P::T* x, double* E,
                             typename P::T* F) {
    const bool acc = (b->flags & NNP_FLAG_ACCUMULATE) != 0;
    hipStream_t st = (hipStream_t)b->stream, st2 = h->st2;
    h->last_stream = st;
    Shape s1 = h->shape, s2 = h->shape;
    const int B1 = b->n_mols / 2;
    s1.A = s2.A = b->n_atoms;   // launch bound of each part
    s1.B = B1;
    s2.B = b->n_mols - B1;
    s1.sub = s2.sub = 1;
    const int32_t* m1 = b->mol_offsets;
    const int32_t* m2 = b->mol_offsets + B1;
    Work<P>& w1 = work_of<P>(h);
    Work<P>& w2 = work2_of<P>(h);
    Timer tm = make_timer(h);
    HIP_TRY(hipEventRecord(h->pev[0], st));
    HIP_TRY(hipStreamWaitEvent(st2, h->pev[0], 0));
    nnp_status rc = stage_features<P>(h, s1, m1, b->species, x, F, acc, w1, st, tm);
    if (rc) return rc;
    HIP_TRY(hipEventRecord(h->pev[1], st));
    HIP_TRY(hipStreamWaitEvent(st2, h->pev[1], 0));
    if ((rc = stage_features<P>(h, s2, m2, b->species, x, F, acc, w2, st2, tm))) return rc;
    HIP_TRY(launch_mlp<P>(s1, weights_of<P>(h), w1, st, tm));
    HIP_TRY(hipEventRecord(h->pev[2], st));
    HIP_TRY(hipStreamWaitEvent(st2, h->pev[2], 0));
    HIP_TRY(launch_mlp<P>(s2, weights_of<P>(h), w2, st2, tm));
    if ((rc = stage_finish<P>(h, s1, m1, b->species, x, E, F, acc, w1, st, tm))) return rc;
    if ((rc = stage_finish<P>(h, s2, m2, b->species, x, E + B1, F, acc, w2, st2, tm))) return rc;
    HIP_TRY(hipEventRecord(h->pev[3], st2));
    HIP_TRY(hipStreamWaitEvent(st, h->pev[3], 0));
    return NNP_OK;
}

template <typename P>
nnp_status run_forward(nnp_handle* h, const nnp_batch* b, const typename P::T* x, double* E,
                       typename P::T* F, typename P::T* aev_out) {
    typedef typename P::T T;
    if (h->shape.pipeline == 2 && h->pipe_ready && !aev_out && b->n_mols >= 2 &&
        !(b->flags & NNP_FLAG_DEVICE_COUNTS))
        return run_forward_split<P>(h, b, x, E, F);
    Shape sh = h->shape;
    launch_bounds(h, b, sh.A, sh.B);
    sh.dev_counts = (b->flags & NNP_FLAG_DEVICE_COUNTS) ? 1 : 0;
    const bool acc = (b->flags & NNP_FLAG_ACCUMULATE) != 0;
    hipStream_t st = (hipStream_t)b->stream;
    h->last_stream = st;
    Work<P>& w = work_of<P>(h);
    const AevConst<T>& c = const_of<T>(h);
    Timer tm = make_timer(h);
    const int32_t* moff = b->mol_offsets;
    if (sh.dev_counts) {
        tm.b("prep", st);
        HIP_TRY(launch_stage_batch(sh.B, sh.A, b->counts, b->mol_offsets, w.moff, w.dcnt, w.flag, st));
        tm.e("prep", st);
        moff = w.moff;
    }
    HIP_TRY(launch_prep_features<P>(sh, c, moff, b->species, x, F, acc, w, aev_out, st, tm));
    const int32_t* sp = elements_of(w, b);
    if (aev_out) return NNP_OK;
    if (sh.A > 0) HIP_TRY(launch_mlp<P>(sh, weights_of<P>(h), w, st, tm));
    const bool fuse_e = F && sh.A > 0 && !sh.force_fixed;
    if (F && sh.A > 0)
        HIP_TRY(launch_forces<P>(sh, c, moff, sp, x, w, F, st, tm,
                                 fuse_e ? energy_args<P>(sh, weights_of<P>(h), w, E, acc) : EnergyArgs<P>()));
    if (!fuse_e)
        HIP_TRY(launch_energy<P>(sh, weights_of<P>(h), moff, sp, w, E, sh.A > 0 ? F : nullptr, acc, st, tm));
    return NNP_OK;
}

// Forward evaluation through the graph cache: replay on a hit; on a miss run
// eagerly (this call's results), then capture the same launch sequence for
// the next calls.  A failed capture leaves the eager result and no entry.
template <typename P>
nnp_status run_forward_graph(nnp_handle* h, const nnp_batch* b, const typename P::T* x, double* E,
                             typename P::T* F) {
    hipStream_t st = (hipStream_t)b->stream;
    const void* key[6] = {b->mol_offsets, b->species, x, E, F, b->counts};
    int kA, kB;
    launch_bounds(h, b, kA, kB);
    for (size_t i = 0; i < h->graphs.size(); ++i)
        if (h->graphs[i].same(kA, kB, b->flags, key, st)) {
            h->last_stream = st;
            HIP_TRY(hipGraphLaunch(h->graphs[i].exec, st));
            ++h->n_replays;
            return NNP_OK;
        }
    nnp_status rc = run_forward<P>(h, b, x, E, F, nullptr);
    if (rc) return rc;
    hipGraph_t graph = nullptr;
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) return NNP_OK;
    rc = run_forward<P>(h, b, x, E, F, nullptr);
    hipError_t e = hipStreamEndCapture(st, &graph);
    if (rc != NNP_OK || e != hipSuccess || !graph) {
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipGetLastError();
        g_err.clear();
        return NNP_OK;
    }
    GraphEntry ge;
    ge.A = kA;
    ge.B = kB;
    ge.flags = b->flags;
    for (int i = 0; i < 6; ++i) ge.ptr[i] = key[i];
    ge.stream = st;
    e = hipGraphInstantiate(&ge.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return NNP_OK;
    if (h->graphs.size() >= kMaxGraphs) {
        (void)hipGraphExecDestroy(h->graphs.front().exec);
        h->graphs.erase(h->graphs.begin());
    }
    h->graphs.push_back(ge);
    ++h->n_captures;
    return NNP_OK;
}

template <typename P> nnp_status alloc_train(nnp_handle* h) {
    typedef typename P::TS TS;
    typedef typename P::T T;
    if (h->train_ready) return NNP_OK;
    TrainWork<P>& tw = train_of<P>(h);
    const Shape& sh = h->shape;
    const size_t R = sh.Rcap;
    const int M = sh.M;
    hipError_t e = hipSuccess;
#define TALLOC(field, bytes)                                                             \
    do {                                                                                 \
        tw.field = (decltype(tw.field))h->dalloc(bytes, e);                              \
        if (e != hipSuccess)                                                             \
            return fail(e == hipErrorOutOfMemory ? NNP_E_NOMEM : NNP_E_DEVICE,           \
                        std::string("training workspace: ") + hipGetErrorString(e));     \
    } while (0)
    TALLOC(GD, sizeof(TS) * R * sh.Dp);
    TALLOC(H3, sizeof(TS) * R * M * sh.H3);
    TALLOC(TH1, sizeof(TS) * R * M * sh.H1);
    TALLOC(TH2, sizeof(TS) * R * M * sh.H2);
    TALLOC(TH3, sizeof(TS) * R * M * sh.H3);
    TALLOC(ZDB1, sizeof(TS) * R * M * sh.H1);
    TALLOC(ZDB2, sizeof(TS) * R * M * sh.H2);
    TALLOC(ZDB3, sizeof(TS) * R * M * sh.H3);
    TALLOC(TMP, sizeof(TS) * R * M * std::max(sh.H1, sh.H2));
#undef TALLOC
    if (h->het) {
        h->gpad = h->dalloc(sizeof(typename P::TA) * (size_t)h->n_int, e);
        if (e != hipSuccess) return fail(NNP_E_NOMEM, "training workspace (padded gradients)");
    }
    h->train_F = h->dalloc(sizeof(T) * 3 * (size_t)std::max(h->max_atoms, 1), e);
    if (e != hipSuccess) return fail(NNP_E_NOMEM, "training workspace (forces)");
    h->train_E = (double*)h->dalloc(sizeof(double) * (size_t)h->max_mols, e);
    if (e != hipSuccess) return fail(NNP_E_NOMEM, "training workspace (energies)");
    // padding rows of the AEV tangent are never written by the featuriser
    HIP_TRY(hipMemset(tw.GD, 0, sizeof(TS) * R * sh.Dp));
    h->train_ready = true;
    return NNP_OK;
}

template <typename P>
nnp_status run_backward(nnp_handle* h, const nnp_batch* bin, const typename P::T* x,
                        const double* gE, const typename P::T* gF, typename P::TA* gp,
                        typename P::T* gx) {
    typedef typename P::T T;
    nnp_status rc = alloc_train<P>(h);
    if (rc) return rc;
    if (bin->flags & NNP_FLAG_DEVICE_COUNTS)
        return fail(NNP_E_UNSUPPORTED, "the training backward takes host counts");
    nnp_batch bb = *bin;   // the internal evaluations overwrite their outputs, eagerly
    bb.flags = 0;
    const nnp_batch* b = &bb;
    Shape sh = h->shape;
    sh.A = b->n_atoms;
    sh.B = b->n_mols;
    sh.force_fixed = 0;    // the force contraction below writes F directly
    hipStream_t st = (hipStream_t)b->stream;
    h->last_stream = st;
    Work<P>& w = work_of<P>(h);
    TrainWork<P>& tw = train_of<P>(h);
    const AevConst<T>& c = const_of<T>(h);
    Timer tm = make_timer(h);
    const bool has_gF = gF != nullptr;
    if (gx && !has_gF) {
        // dL/dx of an energy-only loss: -gE_b F_i from one forward evaluation
        rc = run_forward<P>(h, b, x, h->train_E, (T*)h->train_F, nullptr);
        if (rc) return rc;
        HIP_TRY(launch_grad_coords<P>(sh.A, w.mol_of_atom, gE, (const T*)h->train_F, gx, st));
    }
    if (gx && has_gF) {
        // dL/dx = -gE F - H gF.  With K(r) = -sum_i (dG_i/dx)^T r_i the force
        // contraction of AEV-row cotangents r: H gF = -K(rows' tangent) -
        // (tangent of K(g) along gF at fixed rows g).  Here gx starts as that
        // second tangent, from the forward pass's rows g = dE/dG ...
        rc = run_forward<P>(h, b, x, h->train_E, (T*)h->train_F, nullptr);
        if (rc) return rc;
        HIP_TRY(launch_fill<P>(gx, 3 * (size_t)sh.A, st));
        if (sh.A > 0)
            HIP_TRY(launch_forces_tan<P>(sh, c, b->mol_offsets, elements_of(w, b), x, gF, w, gx, st, tm));
    }
    HIP_TRY(launch_prep<P>(sh, b->mol_offsets, b->species, w, st, tm));
    const int32_t* sp = elements_of(w, b);
    if (sh.A > 0) {
        HIP_TRY(launch_neighbours<P>(sh, c, b->mol_offsets, sp, x, (T*)nullptr, false, w, st, tm));
        HIP_TRY(launch_aev<P>(sh, c, b->mol_offsets, sp, x, w, (T*)nullptr, st, tm));
        if (has_gF)
            HIP_TRY(launch_aev_jvp<P>(sh, c, b->mol_offsets, sp, x, gF, w, tw.GD, st, tm));
    }
    if (!has_gF) {
        // the reverse steps read the tangent activations: make them exact zeros
        const size_t R = sh.Rcap;
        HIP_TRY(launch_fill<P>(tw.TH1, R * sh.M * sh.H1, st));
        HIP_TRY(launch_fill<P>(tw.TH2, R * sh.M * sh.H2, st));
        HIP_TRY(launch_fill<P>(tw.TH3, R * sh.M * sh.H3, st));
    }
    const DevWeights<P>& wt = weights_of<P>(h);
    HIP_TRY(launch_train_mlp<P>(sh, wt, w, tw, w.mol_of_atom, gE, has_gF, st, tm));
    HIP_TRY(launch_train_rev3<P>(sh, wt, w, tw, w.mol_of_atom, gE, has_gF, st, tm));
    HIP_TRY(launch_train_mlp_rev<P>(sh, wt, w, tw, st, tm));
    if (h->het) {
        typedef typename P::TA TA;
        HIP_TRY(launch_train_grads<P>(sh, h->nl, w, tw, w.mol_of_atom, gE, has_gF, (TA*)h->gpad, st, tm));
        HIP_TRY(launch_gather<TA>(h->n_params, h->dmap, (const TA*)h->gpad, gp, st));
    } else {
        HIP_TRY(launch_train_grads<P>(sh, h->nl, w, tw, w.mol_of_atom, gE, has_gF, gp, st, tm));
    }
    if (gx && has_gF && sh.A > 0) {
        // ... and the reverse pass above left DZ1 = the layer-1 adjoint of
        // (u/M)(gE e - edot): its AEV-row adjoint is gE g - gdot, and
        // K(gE g - gdot) = gE F + sum_i (dG_i/dx)^T gdot, so
        // gx = tangent - K(gE g - gdot) = -gE F - H gF.
        HIP_TRY(launch_l1_bwd<P>(sh, weights_of<P>(h), w, st, tm));
        HIP_TRY(launch_fill<P>((T*)h->train_F, 3 * (size_t)sh.A, st));
        HIP_TRY(launch_forces<P>(sh, c, b->mol_offsets, sp, x, w, (T*)h->train_F, st, tm));
        HIP_TRY(launch_sub<T>(3 * (size_t)sh.A, (const T*)h->train_F, gx, st));
    }
    return NNP_OK;
}

// ---------------------------------------------------------------------------
// Autotuner

const char* prec_name(int p) { return p == NNP_PREC_FP64 ? "fp64" : p == NNP_PREC_FP32 ? "fp32" : "bf16"; }
const char* knob_name(int k) {
    return k == NNP_KNOB_MLP_PATH ? "mlp_path"
         : k == NNP_KNOB_GEMM_STAGES ? "gemm_stages"
         : k == NNP_KNOB_CELL_MIN ? "cell_min"
         : k == NNP_KNOB_TAIL_TILE ? "tail_tile"
         : k == NNP_KNOB_GEMM_WAVES ? "gemm_waves"
         : k == NNP_KNOB_ATOM_CHUNK ? "atom_chunk"
         : k == NNP_KNOB_L1_PATH ? "l1_path"
         : k == NNP_KNOB_FORCE_SUM ? "force_sum"
         : k == NNP_KNOB_FORCE_PATH ? "force_path" : "pipeline";
}

std::string tune_key(const nnp_handle* h) {
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, h->device) == hipSuccess) arch = prop.gcnArchName;
    char buf[256];
    std::snprintf(buf, sizeof(buf), "%s|%s|S%d M%d w%d-%d-%d-%d|atoms%d mols%d apm%d", arch.c_str(),
                  prec_name(h->precision), h->S, h->M, h->widths[0], h->widths[1], h->widths[2],
                  h->widths[3], h->max_atoms, h->max_mols, h->max_apm);
    return buf;
}

// integer value of "name": in a flat JSON object, or false if absent
bool json_int(const std::string& line, const char* name, int32_t& v) {
    const std::string pat = std::string("\"") + name + "\":";
    size_t at = line.find(pat);
    if (at == std::string::npos) return false;
    return std::sscanf(line.c_str() + at + pat.size(), " %d", &v) == 1;
}

// look the key up in a JSON-lines cache; fills knobs on a hit
bool cache_lookup(const char* path, const std::string& key, int32_t knobs[NNP_N_KNOBS]) {
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    std::string line;
    bool hit = false;
    char buf[1024];
    while (!hit && std::fgets(buf, sizeof(buf), f)) {
        line = buf;
        if (line.find("\"key\": \"" + key + "\"") == std::string::npos) continue;
        int32_t v[NNP_N_KNOBS];
        bool ok = true;
        for (int k = 0; k < NNP_N_KNOBS; ++k)
            if (k != NNP_KNOB_FORCE_SUM) ok = ok && json_int(line, knob_name(k), v[k]);
        if (ok) {
            for (int k = 0; k < NNP_N_KNOBS; ++k)
                if (k != NNP_KNOB_FORCE_SUM) knobs[k] = v[k];
            hit = true;
        }
    }
    std::fclose(f);
    return hit;
}

template <typename P>
nnp_status time_eval(nnp_handle* h, const nnp_batch* b, const typename P::T* x, double* E,
                     typename P::T* F, int reps, double& us) {
    hipStream_t st = (hipStream_t)b->stream;
    nnp_status rc = run_forward<P>(h, b, x, E, F, nullptr);
    if (rc) return rc;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(NNP_E_DEVICE, "hipEventCreate failed");
    }
    hipError_t e = hipEventRecord(e0, st);
    for (int r = 0; r < reps && rc == NNP_OK && e == hipSuccess; ++r) rc = run_forward<P>(h, b, x, E, F, nullptr);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    if (e != hipSuccess) return fail(NNP_E_DEVICE, std::string("autotune timing: ") + hipGetErrorString(e));
    us = 1e3 * ms / reps;
    return NNP_OK;
}

template <typename P>
nnp_status autotune(nnp_handle* h, const nnp_batch* b, const typename P::T* x, int reps,
                    std::string& timings) {
    typedef typename P::T T;
    hipError_t e = hipSuccess;
    double* E = nullptr;
    T* F = nullptr;
    e = hipMalloc(&E, sizeof(double) * std::max(b->n_mols, 1));
    if (e == hipSuccess) e = hipMalloc(&F, sizeof(T) * 3 * std::max(b->n_atoms, 1));
    nnp_status rc = e == hipSuccess ? NNP_OK : fail(NNP_E_NOMEM, "autotune outputs");
    for (int k = 0; k < NNP_N_KNOBS && rc == NNP_OK; ++k) {
        std::vector<int32_t> cand;
        if (k == NNP_KNOB_MLP_PATH) {
            if (mlp_fused_supported(h->shape.H1, h->shape.H2, h->shape.H3)) cand = {1, 2};
        } else if (k == NNP_KNOB_GEMM_STAGES) {
            cand = {2, 3};
        } else if (k == NNP_KNOB_TAIL_TILE) {
            if (knob_value(h, NNP_KNOB_MLP_PATH) == 1 && h->shape.row_tile == 128) cand = {1, 2, 3};
        } else if (k == NNP_KNOB_GEMM_WAVES) {
            if (h->shape.row_tile == 128 && h->precision != NNP_PREC_FP64) cand = {4, 8};
        } else if (k == NNP_KNOB_ATOM_CHUNK) {
            cand = {4, 8, 16};
        } else if (k == NNP_KNOB_L1_PATH) {
            if (l1_regs_supported(h)) cand = {1, 2};
        } else if (k == NNP_KNOB_FORCE_SUM) {
            // reproducibility is the caller's choice: never tuned
        } else if (k == NNP_KNOB_FORCE_PATH) {
            cand = {1, 2};
        } else if (k == NNP_KNOB_PIPELINE) {
            if (h->max_mols >= 2) cand = {1, 2};
        } else {
            for (int c : {32, 64, 128, 256})
                if (c < h->max_apm) cand.push_back(c);
            if (!cand.empty()) cand.push_back(1024);
        }
        if (cand.size() < 2) {
            h->knob[k] = knob_value(h, k);
            continue;
        }
        double best = 1e300;
        int32_t best_v = cand[0];
        for (int32_t v : cand) {
            h->knob[k] = v;
            apply_knobs(h);
            if ((rc = ensure_pipeline(h))) break;
            double us = 0;
            rc = time_eval<P>(h, b, x, E, F, reps, us);
            if (rc) break;
            char buf[96];
            std::snprintf(buf, sizeof(buf), "%s\"%s=%d\": %.2f", timings.empty() ? "" : ", ",
                          knob_name(k), v, us);
            timings += buf;
            if (us < best) {
                best = us;
                best_v = v;
            }
        }
        h->knob[k] = best_v;
        apply_knobs(h);
    }
    if (E) (void)hipFree(E);
    if (F) (void)hipFree(F);
    return rc;
}

}  // namespace

// ===========================================================================
extern "C" {

const char* nnp_last_error(void) { return g_err.c_str(); }

nnp_status nnp_create(const nnp_model_params* p, nnp_handle** out) {
    if (!out) return fail(NNP_E_INVALID, "null output pointer");
    *out = nullptr;
    if (!p) return fail(NNP_E_INVALID, "null params");
    if (p->n_species < 1 || p->n_species > NNP_MAX_SPECIES)
        return fail(NNP_E_INVALID, "n_species must be in 1..8");
    if (!p->shf_r || !p->shf_a || !p->shf_z || !p->weights || (!p->widths && !p->species_widths))
        return fail(NNP_E_INVALID, "null shift, width or weight array");
    if (p->n_shf_r != kNR || p->n_shf_a * p->n_shf_z != kNAZ || (p->n_shf_z != 4 && p->n_shf_z != 8))
        return fail(NNP_E_UNSUPPORTED, "the library supports 16 radial shifts and 8x4 or 4x8 angular shifts");
    if (!(p->rcr > 0) || !(p->rca > 0) || p->rca > p->rcr)
        return fail(NNP_E_INVALID, "cutoffs must satisfy 0 < rca <= rcr");
    if (!(p->angle_scale > 0 && p->angle_scale < 1))
        return fail(NNP_E_INVALID, "angle_scale must be in (0, 1)");
    if (!(p->zeta >= 1) || !(p->eta_r >= 0) || !(p->eta_a >= 0))
        return fail(NNP_E_INVALID, "need zeta >= 1, eta_r >= 0, eta_a >= 0");
    if (!(p->celu_alpha > 0)) return fail(NNP_E_INVALID, "celu_alpha must be > 0");
    if (p->n_models < 1 || p->n_models > 64) return fail(NNP_E_INVALID, "n_models must be in 1..64");
    if (p->n_layers != 4) return fail(NNP_E_UNSUPPORTED, "the library supports 4 affine layers");
    const int S = p->n_species;
    const int D = S * p->n_shf_r + (S * (S + 1) / 2) * p->n_shf_a * p->n_shf_z;
    // element network widths sw[s][l]; the uniform layout wi[l] every element
    // network is padded to (the widest, rounded up to a multiple of 32)
    std::vector<int> sw((size_t)S * 5), wi(5, 0);
    for (int s = 0; s < S; ++s)
        for (int l = 0; l < 5; ++l) sw[s * 5 + l] = p->species_widths ? p->species_widths[s * 5 + l] : p->widths[l];
    for (int s = 0; s < S; ++s) {
        const int* ws = &sw[s * 5];
        if (ws[0] != D) return fail(NNP_E_INVALID, "widths[0] must equal the AEV dimension");
        if (ws[4] != 1) return fail(NNP_E_INVALID, "the last width must be 1");
        for (int l = 1; l < 4; ++l) {
            if (ws[l] < 1 || ws[l] > 4096) return fail(NNP_E_UNSUPPORTED, "hidden widths must be in 1..4096");
            if (!p->species_widths && ws[l] % 32)
                return fail(NNP_E_UNSUPPORTED, "hidden widths must be multiples of 32 up to 4096");
        }
    }
    wi[0] = D;
    wi[4] = 1;
    for (int l = 1; l < 4; ++l)
        for (int s = 0; s < S; ++s) wi[l] = std::max(wi[l], pad_to(sw[s * 5 + l], 32));
    if (p->precision < NNP_PREC_FP64 || p->precision > NNP_PREC_BF16_MLP)
        return fail(NNP_E_INVALID, "unknown precision");
    if (p->max_atoms < 1 || p->max_mols < 1 || p->max_atoms_per_mol < 1)
        return fail(NNP_E_INVALID, "capacities must be >= 1");
    if (p->max_atoms_per_mol > kMaxAtomsPerMol)
        return fail(NNP_E_UNSUPPORTED, "max_atoms_per_mol is limited to 1024");
    if (p->max_atoms > (1 << 26)) return fail(NNP_E_INVALID, "max_atoms too large");
    if (p->create_flags & ~NNP_CREATE_TRAINING) return fail(NNP_E_INVALID, "unknown creation flags");
    if ((p->create_flags & NNP_CREATE_TRAINING) && p->precision == NNP_PREC_BF16_MLP)
        return fail(NNP_E_UNSUPPORTED, "the training backward runs on FP32 or FP64 handles");
    // element table: atomic number -> element index
    std::vector<int8_t> lut;
    if (p->atomic_numbers) {
        lut.assign(kZLut, -1);
        for (int s = 0; s < S; ++s) {
            const int z = p->atomic_numbers[s];
            if (z < 1 || z >= kZLut) return fail(NNP_E_SPECIES, "atomic numbers must be in 1..127");
            if (lut[z] >= 0) return fail(NNP_E_SPECIES, "atomic number listed twice in the element table");
            lut[z] = (int8_t)s;
        }
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
        return fail(NNP_E_DEVICE, "no HIP device available");
    if (p->device < 0 || p->device >= ndev) return fail(NNP_E_INVALID, "device ordinal out of range");

    nnp_handle* h = new nnp_handle();
    h->S = S;
    h->nR = p->n_shf_r;
    h->nA = p->n_shf_a;
    h->nZ = p->n_shf_z;
    h->D = D;
    h->M = p->n_models;
    h->L = p->n_layers;
    h->widths = wi;
    h->het = p->species_widths != nullptr;
    h->precision = p->precision;
    h->device = p->device;
    h->max_atoms = p->max_atoms;
    h->max_mols = p->max_mols;
    h->max_apm = std::min(p->max_atoms_per_mol, p->max_atoms);
    h->energy_scale = p->energy_scale;
    h->celu_alpha = p->celu_alpha;
    if (p->sae) h->sae.assign(p->sae, p->sae + S);
    auto net_of = [](const int* w) {
        int64_t n = 0;
        for (int l = 0; l < 4; ++l) n += (int64_t)w[l + 1] * w[l] + w[l + 1];
        return n;
    };
    const int64_t net_int = net_of(wi.data());
    h->n_int = net_int * S * h->M;
    h->n_params = 0;
    for (int s = 0; s < S; ++s) h->n_params += net_of(&sw[s * 5]) * h->M;
    if (h->het) {
        if (h->n_int >= ((int64_t)1 << 31)) {
            delete h;
            return fail(NNP_E_UNSUPPORTED, "padded parameter count above 2^31");
        }
        // packed index -> padded index, layer by layer: W row-major, then b
        h->pmap.reserve((size_t)h->n_params);
        for (int m = 0; m < h->M; ++m)
            for (int s = 0; s < S; ++s) {
                const int* ws = &sw[s * 5];
                int64_t base = ((int64_t)m * S + s) * net_int;
                for (int l = 0; l < 4; ++l) {
                    for (int n = 0; n < ws[l + 1]; ++n)
                        for (int k = 0; k < ws[l]; ++k) h->pmap.push_back((int32_t)(base + (int64_t)n * wi[l] + k));
                    for (int n = 0; n < ws[l + 1]; ++n)
                        h->pmap.push_back((int32_t)(base + (int64_t)wi[l + 1] * wi[l] + n));
                    base += (int64_t)wi[l + 1] * wi[l] + wi[l + 1];
                }
            }
    }
    {
        NetLayout& nl = h->nl;
        nl.D = D;
        nl.o1 = wi[1];
        nl.o2 = wi[2];
        nl.o3 = wi[3];
        nl.offW1 = 0;
        nl.offb1 = (long)nl.o1 * D;
        nl.offW2 = nl.offb1 + nl.o1;
        nl.offb2 = nl.offW2 + (long)nl.o2 * nl.o1;
        nl.offW3 = nl.offb2 + nl.o2;
        nl.offb3 = nl.offW3 + (long)nl.o3 * nl.o2;
        nl.offw4 = nl.offb3 + nl.o3;
        nl.offb4 = nl.offw4 + nl.o3;
        nl.net = nl.offb4 + 1;
    }

    Shape& sh = h->shape;
    sh.S = S;
    sh.M = h->M;
    sh.D = D;
    sh.Dp = pad_to(D, 64);
    sh.H1 = pad_to(wi[1], 64);
    sh.H2 = pad_to(wi[2], 64);
    sh.H3 = pad_to(wi[3], 64);
    sh.h3_used = wi[3];
    sh.row_tile = (p->max_atoms <= 256 || p->precision == NNP_PREC_FP64) ? 16 : 128;
    sh.Rcap = pad_to(p->max_atoms + S * (sh.row_tile - 1), sh.row_tile);
    sh.cap_nbr = std::max(1, std::min(h->max_apm - 1, kMaxNeighbours));
    sh.max_apm = h->max_apm;
    sh.energy_scale = p->energy_scale;
    sh.celu_alpha = p->celu_alpha;
    apply_knobs(h);
    fill_const(h->cf, p, D, sh.Dp);
    fill_const(h->cd, p, D, sh.Dp);

    DeviceGuard dg(h->device);
    if (!dg.ok) {
        delete h;
        return fail(NNP_E_DEVICE, "hipSetDevice failed");
    }
    hipError_t e = hipSuccess;
    h->flag = (int32_t*)h->dalloc(sizeof(int32_t), e);
    nnp_status rc = e == hipSuccess ? NNP_OK : fail(NNP_E_NOMEM, "flag allocation failed");
    if (rc == NNP_OK && hipMemset(h->flag, 0, sizeof(int32_t)) != hipSuccess)
        rc = fail(NNP_E_DEVICE, "hipMemset failed");
    if (rc == NNP_OK && !lut.empty()) {
        h->zlut = (int8_t*)h->dalloc(kZLut, e);
        if (e != hipSuccess)
            rc = fail(NNP_E_NOMEM, "element table allocation failed");
        else if (hipMemcpy(h->zlut, lut.data(), kZLut, hipMemcpyHostToDevice) != hipSuccess)
            rc = fail(NNP_E_DEVICE, "element table upload failed");
    }
    if (rc == NNP_OK && h->het) {
        h->dmap = (int32_t*)h->dalloc(sizeof(int32_t) * h->pmap.size(), e);
        if (e != hipSuccess)
            rc = fail(NNP_E_NOMEM, "parameter map allocation failed");
        else if (hipMemcpy(h->dmap, h->pmap.data(), sizeof(int32_t) * h->pmap.size(), hipMemcpyHostToDevice) != hipSuccess)
            rc = fail(NNP_E_DEVICE, "parameter map upload failed");
    }
    if (rc == NNP_OK) {
        if (p->precision == NNP_PREC_FP64) {
            rc = upload_weights<PrecF64>(h, h->w64, p->weights, true);
            if (rc == NNP_OK) rc = alloc_work<PrecF64>(h, h->k64);
        } else if (p->precision == NNP_PREC_FP32) {
            rc = upload_weights<PrecF32>(h, h->w32, p->weights, true);
            if (rc == NNP_OK) rc = alloc_work<PrecF32>(h, h->k32);
        } else {
            rc = upload_weights<PrecBF16>(h, h->w16, p->weights, true);
            if (rc == NNP_OK) rc = alloc_work<PrecBF16>(h, h->k16);
        }
    }
    if (rc == NNP_OK) rc = ensure_pipeline(h);
    if (rc == NNP_OK && (p->create_flags & NNP_CREATE_TRAINING))
        rc = p->precision == NNP_PREC_FP64 ? alloc_train<PrecF64>(h) : alloc_train<PrecF32>(h);
    if (rc != NNP_OK) {
        std::string msg = g_err;
        nnp_destroy(h);
        g_err = msg;
        return rc;
    }
    *out = h;
    return NNP_OK;
}

void nnp_destroy(nnp_handle* h) {
    if (!h) return;
    DeviceGuard dg(h->device);
    (void)hipDeviceSynchronize();
    for (void* p : h->allocs) (void)hipFree(p);
    for (auto& p : h->pending) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (auto e : h->free_events) (void)hipEventDestroy(e);
    for (auto& g : h->graphs) (void)hipGraphExecDestroy(g.exec);
    for (auto e : h->pev)
        if (e) (void)hipEventDestroy(e);
    if (h->st2) (void)hipStreamDestroy(h->st2);
    delete h;
}

nnp_status nnp_energy_forces(nnp_handle* h, const nnp_batch* b, const float* coords,
                             double* out_E, float* out_F) {
    nnp_status rc = check_batch(h, b);
    if (rc) return rc;
    if (h->precision == NNP_PREC_FP64)
        return fail(NNP_E_INVALID, "FP64 handle: use nnp_energy_forces_f64");
    if (!out_E || (b->n_atoms > 0 && !coords)) return fail(NNP_E_INVALID, "null coords or out_E");
    DeviceGuard dg(h->device);
    if (!dg.ok) return fail(NNP_E_DEVICE, "hipSetDevice failed");
    const bool graph = (b->flags & NNP_FLAG_GRAPH) && !h->timing;
    if (h->precision == NNP_PREC_FP32)
        return graph ? run_forward_graph<PrecF32>(h, b, coords, out_E, out_F)
                     : run_forward<PrecF32>(h, b, coords, out_E, out_F, nullptr);
    return graph ? run_forward_graph<PrecBF16>(h, b, coords, out_E, out_F)
                 : run_forward<PrecBF16>(h, b, coords, out_E, out_F, nullptr);
}

nnp_status nnp_energy_forces_f64(nnp_handle* h, const nnp_batch* b, const double* coords,
                                 double* out_E, double* out_F) {
    nnp_status rc = check_batch(h, b);
    if (rc) return rc;
    if (h->precision != NNP_PREC_FP64)
        return fail(NNP_E_INVALID, "FP32/BF16 handle: use nnp_energy_forces");
    if (!out_E || (b->n_atoms > 0 && !coords)) return fail(NNP_E_INVALID, "null coords or out_E");
    DeviceGuard dg(h->device);
    if (!dg.ok) return fail(NNP_E_DEVICE, "hipSetDevice failed");
    if ((b->flags & NNP_FLAG_GRAPH) && !h->timing)
        return run_forward_graph<PrecF64>(h, b, coords, out_E, out_F);
    return run_forward<PrecF64>(h, b, coords, out_E, out_F, nullptr);
}

nnp_status nnp_aev(nnp_handle* h, const nnp_batch* b, const void* coords, void* out_aev) {
    nnp_status rc = check_batch(h, b);
    if (rc) return rc;
    if (b->flags & NNP_FLAG_DEVICE_COUNTS) return fail(NNP_E_UNSUPPORTED, "nnp_aev takes host counts");
    if (!out_aev || (b->n_atoms > 0 && !coords)) return fail(NNP_E_INVALID, "null coords or out_aev");
    DeviceGuard dg(h->device);
    if (!dg.ok) return fail(NNP_E_DEVICE, "hipSetDevice failed");
    if (h->precision == NNP_PREC_FP64)
        return run_forward<PrecF64>(h, b, (const double*)coords, nullptr, nullptr, (double*)out_aev);
    if (h->precision == NNP_PREC_FP32)
        return run_forward<PrecF32>(h, b, (const float*)coords, nullptr, nullptr, (float*)out_aev);
    return run_forward<PrecBF16>(h, b, (const float*)coords, nullptr, nullptr, (float*)out_aev);
}

nnp_status nnp_energy_forces_backward(nnp_handle* h, const nnp_batch* b, const void* coords,
                                      const double* grad_E, const void* grad_F,
                                      void* grad_params, void* grad_coords) {
    nnp_status rc = check_batch(h, b);
    if (rc) return rc;
    if (!grad_params || (b->n_atoms > 0 && !coords))
        return fail(NNP_E_INVALID, "null coords or grad_params");
    if (h->precision == NNP_PREC_BF16_MLP)
        return fail(NNP_E_UNSUPPORTED, "the training backward runs on FP32 or FP64 handles");
    DeviceGuard dg(h->device);
    if (!dg.ok) return fail(NNP_E_DEVICE, "hipSetDevice failed");
    if (h->precision == NNP_PREC_FP64)
        return run_backward<PrecF64>(h, b, (const double*)coords, grad_E, (const double*)grad_F,
                                     (double*)grad_params, (double*)grad_coords);
    return run_backward<PrecF32>(h, b, (const float*)coords, grad_E, (const float*)grad_F,
                                 (float*)grad_params, (float*)grad_coords);
}

nnp_status nnp_set_weights(nnp_handle* h, const double* weights) {
    if (!h || !weights) return fail(NNP_E_INVALID, "null handle or weights");
    DeviceGuard dg(h->device);
    if (!dg.ok) return fail(NNP_E_DEVICE, "hipSetDevice failed");
    HIP_TRY(hipDeviceSynchronize());
    if (h->precision == NNP_PREC_FP64) return upload_weights<PrecF64>(h, h->w64, weights, false);
    if (h->precision == NNP_PREC_FP32) return upload_weights<PrecF32>(h, h->w32, weights, false);
    return upload_weights<PrecBF16>(h, h->w16, weights, false);
}

nnp_status nnp_set_params(nnp_handle* h, const void* params, int32_t type, void* stream) {
    if (!h || !params) return fail(NNP_E_INVALID, "null handle or params");
    if (type != NNP_PREC_FP64 && type != NNP_PREC_FP32)
        return fail(NNP_E_INVALID, "parameter type must be NNP_PREC_FP64 or NNP_PREC_FP32");
    DeviceGuard dg(h->device);
    if (!dg.ok) return fail(NNP_E_DEVICE, "hipSetDevice failed");
    const NetLayout& nl = h->nl;
    ParamPack pk{};
    pk.S = h->S;
    pk.M = h->M;
    pk.D = h->D;
    pk.Dp = h->shape.Dp;
    pk.H1 = h->shape.H1;
    pk.H2 = h->shape.H2;
    pk.H3 = h->shape.H3;
    pk.o1 = nl.o1;
    pk.o2 = nl.o2;
    pk.net = nl.net;
    pk.offb1 = nl.offb1;
    pk.offW2 = nl.offW2;
    pk.offb2 = nl.offb2;
    pk.offW3 = nl.offW3;
    pk.offb3 = nl.offb3;
    pk.offw4 = nl.offw4;
    pk.offb4 = nl.offb4;
    const int32_t* map = h->het ? h->dmap : nullptr;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e;
    if (h->precision == NNP_PREC_FP64)
        e = type == NNP_PREC_FP64 ? launch_set_params<PrecF64>(h->n_params, (const double*)params, map, pk, h->w64, st)
                                  : launch_set_params<PrecF64>(h->n_params, (const float*)params, map, pk, h->w64, st);
    else if (h->precision == NNP_PREC_FP32)
        e = type == NNP_PREC_FP64 ? launch_set_params<PrecF32>(h->n_params, (const double*)params, map, pk, h->w32, st)
                                  : launch_set_params<PrecF32>(h->n_params, (const float*)params, map, pk, h->w32, st);
    else
        e = type == NNP_PREC_FP64 ? launch_set_params<PrecBF16>(h->n_params, (const double*)params, map, pk, h->w16, st)
                                  : launch_set_params<PrecBF16>(h->n_params, (const float*)params, map, pk, h->w16, st);
    if (e != hipSuccess) return fail(NNP_E_DEVICE, std::string("parameter update: ") + hipGetErrorString(e));
    return NNP_OK;
}

int64_t nnp_num_params(const nnp_handle* h) { return h ? h->n_params : -1; }

nnp_status nnp_graph_stats(const nnp_handle* h, int64_t* captures, int64_t* replays, int32_t* cached) {
    if (!h) return fail(NNP_E_INVALID, "null handle");
    if (captures) *captures = h->n_captures;
    if (replays) *replays = h->n_replays;
    if (cached) *cached = (int32_t)h->graphs.size();
    return NNP_OK;
}

int32_t nnp_aev_dim(const nnp_handle* h) { return h ? h->D : -1; }

nnp_status nnp_get_device_status(nnp_handle* h, int32_t* code) {
    if (!h || !code) return fail(NNP_E_INVALID, "null handle or code");
    DeviceGuard dg(h->device);
    if (!dg.ok) return fail(NNP_E_DEVICE, "hipSetDevice failed");
    HIP_TRY(hipStreamSynchronize(h->last_stream));
    int32_t f = 0;
    HIP_TRY(hipMemcpy(&f, h->flag, sizeof(f), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemset(h->flag, 0, sizeof(int32_t)));
    *code = (f & FLAG_SPECIES) ? NNP_E_SPECIES : (f & FLAG_CAPACITY) ? NNP_E_CAPACITY : NNP_OK;
    return NNP_OK;
}

nnp_status nnp_set_timing(nnp_handle* h, int32_t enable) {
    if (!h) return fail(NNP_E_INVALID, "null handle");
    DeviceGuard dg(h->device);
    for (auto& p : h->pending) {
        (void)hipEventSynchronize(p.b);
        h->free_events.push_back(p.a);
        h->free_events.push_back(p.b);
    }
    h->pending.clear();
    h->totals.clear();
    h->timing = enable != 0;
    return NNP_OK;
}

nnp_status nnp_set_timing_only(nnp_handle* h, const char* name) {
    if (!h) return fail(NNP_E_INVALID, "null handle");
    const nnp_status rc = nnp_set_timing(h, h->timing ? 1 : 0);   // clears the totals
    if (rc != NNP_OK) return rc;
    h->timing_only = name ? name : "";
    return NNP_OK;
}

int32_t nnp_kernel_times(nnp_handle* h, int32_t cap, const char** names, int64_t* counts,
                         double* total_ms) {
    if (!h) return -1;
    DeviceGuard dg(h->device);
    for (auto& p : h->pending) {
        (void)hipEventSynchronize(p.b);
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            auto& t = h->totals[p.name];
            t.first += 1;
            t.second += ms;
        }
        h->free_events.push_back(p.a);
        h->free_events.push_back(p.b);
    }
    h->pending.clear();
    int32_t n = 0;
    for (auto& kv : h->totals) {
        if (n < cap) {
            // names point into static storage of the launchers (string literals)
            static thread_local std::vector<std::string> keep;
            if ((int)keep.size() < cap) keep.resize(cap);
            keep[n] = kv.first;
            if (names) names[n] = keep[n].c_str();
            if (counts) counts[n] = kv.second.first;
            if (total_ms) total_ms[n] = kv.second.second;
        }
        ++n;
    }
    return n;
}

nnp_status nnp_set_knob(nnp_handle* h, int32_t knob, int32_t value) {
    if (!h) return fail(NNP_E_INVALID, "null handle");
    if (knob < 0 || knob >= NNP_N_KNOBS) return fail(NNP_E_INVALID, "unknown knob");
    bool ok = value == 0;
    if (knob == NNP_KNOB_MLP_PATH) {
        if (value == 1 && !mlp_fused_supported(h->shape.H1, h->shape.H2, h->shape.H3))
            return fail(NNP_E_UNSUPPORTED, "the fused layers 2-3 kernel needs hidden widths 256-192-(160..192)");
        ok = ok || value == 1 || value == 2;
    } else if (knob == NNP_KNOB_GEMM_STAGES) {
        ok = ok || value == 2 || value == 3;
    } else if (knob == NNP_KNOB_TAIL_TILE) {
        ok = ok || (value >= 1 && value <= 3);
    } else if (knob == NNP_KNOB_GEMM_WAVES) {
        ok = ok || value == 4 || value == 8;
    } else if (knob == NNP_KNOB_ATOM_CHUNK) {
        ok = ok || value == 4 || value == 8 || value == 16;
    } else if (knob == NNP_KNOB_L1_PATH) {
        if (value == 2 && !l1_regs_supported(h))
            return fail(NNP_E_UNSUPPORTED, "register-operand layer-1 GEMMs need BF16 and 128-row buckets");
        ok = ok || value == 1 || value == 2;
    } else if (knob == NNP_KNOB_FORCE_SUM) {
        ok = ok || value == 1 || value == 2;
    } else if (knob == NNP_KNOB_FORCE_PATH || knob == NNP_KNOB_PIPELINE) {
        ok = ok || value == 1 || value == 2;
    } else {
        ok = ok || (value >= 16 && value <= kMaxAtomsPerMol);
    }
    if (!ok) return fail(NNP_E_INVALID, "knob value out of range");
    DeviceGuard dg(h->device);
    if (!h->graphs.empty()) (void)hipDeviceSynchronize();
    h->knob[knob] = value;
    apply_knobs(h);
    return ensure_pipeline(h);
}

nnp_status nnp_get_knob(nnp_handle* h, int32_t knob, int32_t* value) {
    if (!h || !value) return fail(NNP_E_INVALID, "null handle or value");
    if (knob < 0 || knob >= NNP_N_KNOBS) return fail(NNP_E_INVALID, "unknown knob");
    *value = knob_value(h, knob);
    return NNP_OK;
}

nnp_status nnp_autotune(nnp_handle* h, const nnp_batch* b, const void* coords, int32_t reps,
                        const char* cache_path, char* report, int32_t report_cap) {
    nnp_status rc = check_batch(h, b);
    if (rc) return rc;
    if (b->flags & NNP_FLAG_DEVICE_COUNTS) return fail(NNP_E_UNSUPPORTED, "the autotuner takes host counts");
    if (reps < 1 || reps > 1000) return fail(NNP_E_INVALID, "reps must be in 1..1000");
    if (b->n_atoms > 0 && !coords) return fail(NNP_E_INVALID, "null coords");
    DeviceGuard dg(h->device);
    if (!dg.ok) return fail(NNP_E_DEVICE, "hipSetDevice failed");
    const std::string key = tune_key(h);
    int32_t cached[NNP_N_KNOBS];
    bool hit = cache_path && cache_lookup(cache_path, key, cached);
    std::string timings;
    if (hit) {
        if (!h->graphs.empty()) (void)hipDeviceSynchronize();
        for (int k = 0; k < NNP_N_KNOBS; ++k)
            if (k != NNP_KNOB_FORCE_SUM) h->knob[k] = cached[k];
        apply_knobs(h);
        if ((rc = ensure_pipeline(h))) return rc;
    } else {
        if (!h->graphs.empty()) (void)hipDeviceSynchronize();
        if (h->precision == NNP_PREC_FP64)
            rc = autotune<PrecF64>(h, b, (const double*)coords, reps, timings);
        else if (h->precision == NNP_PREC_FP32)
            rc = autotune<PrecF32>(h, b, (const float*)coords, reps, timings);
        else
            rc = autotune<PrecBF16>(h, b, (const float*)coords, reps, timings);
        if (rc) return rc;
    }
    std::string vals;
    for (int k = 0; k < NNP_N_KNOBS; ++k)
        vals += std::string(k ? ", " : "") + "\"" + knob_name(k) + "\": " + std::to_string(knob_value(h, k));
    if (!hit && cache_path) {
        FILE* f = std::fopen(cache_path, "a");
        if (!f) return fail(NNP_E_INVALID, std::string("cannot append to tune cache ") + cache_path);
        std::fprintf(f, "{\"key\": \"%s\", %s}\n", key.c_str(), vals.c_str());
        std::fclose(f);
    }
    if (report && report_cap > 0) {
        std::string r = "{\"key\": \"" + key + "\", \"cached\": " + (hit ? "true" : "false") +
                        ", \"chosen\": {" + vals + "}, \"timings_us\": {" + timings + "}}";
        std::snprintf(report, (size_t)report_cap, "%s", r.c_str());
    }
    return NNP_OK;
}

// ---------------------------------------------------------------------------
// NNP-MM coupling

}  // extern "C"

namespace {
// MM atoms per NNP-side wave: 16, widened (up to 512, the LDS limit of four
// FP64 chunks) by 16 per 64k MM atoms so the partials stay bounded
int coupling_chunk(int max_mm) {
    return 16 * std::min(32, std::max(1, (max_mm + 64 * 1024 - 1) / (64 * 1024)));
}

nnp_status check_coupling_args(int32_t n_nnp, const void* x_nnp, const void* par_nnp, int32_t n_mm,
                               const void* x_mm, const void* par_mm, const double* out_E,
                               const void* F_nnp, const void* F_mm, uint32_t flags) {
    if (!out_E) return fail(NNP_E_INVALID, "null out_E");
    if (n_nnp < 0 || n_mm < 0) return fail(NNP_E_INVALID, "negative atom count");
    if (n_nnp > 0 && (!x_nnp || !par_nnp || !F_nnp)) return fail(NNP_E_INVALID, "null NNP array");
    if (n_mm > 0 && (!x_mm || !par_mm || !F_mm)) return fail(NNP_E_INVALID, "null MM array");
    if (flags & ~NNP_FLAG_ACCUMULATE) return fail(NNP_E_INVALID, "unknown flag");
    return NNP_OK;
}
}  // namespace

struct nnp_coupling {
    nnp::CouplingShape cs{};
    int precision = NNP_PREC_FP32;
    int device = 0;
    double* e_part = nullptr;   // [ceil(max_mm / 256)]
    void* f_part = nullptr;     // [ceil(max_mm / chunk)][max_nnp][3]
};

extern "C" {

nnp_status nnp_coupling_create(int32_t precision, int32_t max_nnp, int32_t max_mm, double coulomb_k,
                               double cutoff, int32_t device, nnp_coupling** out) {
    if (!out) return fail(NNP_E_INVALID, "null output pointer");
    *out = nullptr;
    if (precision != NNP_PREC_FP64 && precision != NNP_PREC_FP32)
        return fail(NNP_E_INVALID, "coupling precision must be FP64 or FP32");
    if (max_nnp < 1 || max_nnp > 1024) return fail(NNP_E_INVALID, "max_nnp must be in 1..1024");
    if (max_mm < 1 || max_mm > (1 << 22)) return fail(NNP_E_INVALID, "max_mm must be in 1..2^22");
    if (!std::isfinite(coulomb_k) || !(cutoff >= 0.0) || !std::isfinite(cutoff))
        return fail(NNP_E_INVALID, "coulomb_k must be finite and cutoff >= 0");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(NNP_E_DEVICE, "no HIP device available");
    if (device < 0 || device >= ndev) return fail(NNP_E_INVALID, "device ordinal out of range");
    DeviceGuard dg(device);
    if (!dg.ok) return fail(NNP_E_DEVICE, "hipSetDevice failed");
    nnp_coupling* c = new nnp_coupling();
    c->precision = precision;
    c->device = device;
    c->cs.coulomb_k = coulomb_k;
    c->cs.cutoff = cutoff;
    c->cs.max_nnp = max_nnp;
    c->cs.max_mm = max_mm;
    c->cs.chunk = coupling_chunk(max_mm);
    const size_t tsz = precision == NNP_PREC_FP64 ? sizeof(double) : sizeof(float);
    const size_t n_eblk = (size_t)(max_mm + kCoupleMmPerBlock - 1) / kCoupleMmPerBlock;
    const size_t n_chunks = (size_t)(max_mm + c->cs.chunk - 1) / c->cs.chunk;
    hipError_t e = hipMalloc(&c->e_part, sizeof(double) * n_eblk);
    if (e == hipSuccess) e = hipMalloc(&c->f_part, tsz * 3 * n_chunks * (size_t)max_nnp);
    if (e != hipSuccess) {
        nnp_coupling_destroy(c);
        return fail(NNP_E_NOMEM, "coupling workspace allocation failed");
    }
    *out = c;
    return NNP_OK;
}

void nnp_coupling_destroy(nnp_coupling* c) {
    if (!c) return;
    DeviceGuard dg(c->device);
    (void)hipDeviceSynchronize();
    if (c->e_part) (void)hipFree(c->e_part);
    if (c->f_part) (void)hipFree(c->f_part);
    delete c;
}

nnp_status nnp_coupling_eval(nnp_coupling* c, int32_t n_nnp, const void* x_nnp, const void* par_nnp,
                             int32_t n_mm, const void* x_mm, const void* par_mm, double* out_E,
                             void* F_nnp, void* F_mm, void* stream, uint32_t flags) {
    if (!c) return fail(NNP_E_INVALID, "null coupling handle");
    nnp_status rc = check_coupling_args(n_nnp, x_nnp, par_nnp, n_mm, x_mm, par_mm, out_E, F_nnp, F_mm, flags);
    if (rc) return rc;
    if (n_nnp > c->cs.max_nnp || n_mm > c->cs.max_mm)
        return fail(NNP_E_CAPACITY, "coupling system exceeds the capacity given at creation");
    DeviceGuard dg(c->device);
    if (!dg.ok) return fail(NNP_E_DEVICE, "hipSetDevice failed");
    const bool acc = (flags & NNP_FLAG_ACCUMULATE) != 0;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e;
    if (c->precision == NNP_PREC_FP64)
        e = launch_coupling<double>(c->cs, n_nnp, (const double*)x_nnp, (const double*)par_nnp, n_mm,
                                    (const double*)x_mm, (const double*)par_mm, out_E, (double*)F_nnp,
                                    (double*)F_mm, c->e_part, (double*)c->f_part, acc, st);
    else
        e = launch_coupling<float>(c->cs, n_nnp, (const float*)x_nnp, (const float*)par_nnp, n_mm,
                                   (const float*)x_mm, (const float*)par_mm, out_E, (float*)F_nnp,
                                   (float*)F_mm, c->e_part, (float*)c->f_part, acc, st);
    if (e != hipSuccess) return fail(NNP_E_DEVICE, std::string("coupling launch: ") + hipGetErrorString(e));
    return NNP_OK;
}

nnp_status nnp_coupling_eval_noalloc(int32_t precision, double coulomb_k, double cutoff, int32_t n_nnp,
                                     const void* x_nnp, const void* par_nnp, int32_t n_mm,
                                     const void* x_mm, const void* par_mm, double* out_E, void* F_nnp,
                                     void* F_mm, void* stream, uint32_t flags) {
    if (precision != NNP_PREC_FP64 && precision != NNP_PREC_FP32)
        return fail(NNP_E_INVALID, "coupling precision must be FP64 or FP32");
    if (!std::isfinite(coulomb_k) || !(cutoff >= 0.0) || !std::isfinite(cutoff))
        return fail(NNP_E_INVALID, "coulomb_k must be finite and cutoff >= 0");
    nnp_status rc = check_coupling_args(n_nnp, x_nnp, par_nnp, n_mm, x_mm, par_mm, out_E, F_nnp, F_mm, flags);
    if (rc) return rc;
    if (n_nnp > 1024 || n_mm > (1 << 22))
        return fail(NNP_E_CAPACITY, "coupling system above 1024 NNP or 2^22 MM atoms");
    void* scratch = nullptr;
    hipError_t e = coupling_scratch(&scratch);
    if (e != hipSuccess) return fail(NNP_E_DEVICE, std::string("coupling scratch: ") + hipGetErrorString(e));
    // the partials: [ceil(n_mm / 64)] doubles, then [3 n_nnp][ceil(n_mm / chunk)]
    // of the operand type; a chunk wider than the handle's rule (up to 512 MM
    // atoms) is taken when that makes them fit
    const size_t tsz = precision == NNP_PREC_FP64 ? sizeof(double) : sizeof(float);
    const size_t e_bytes = (((size_t)(n_mm + kCoupleMmPerBlock - 1) / kCoupleMmPerBlock) * sizeof(double) + 255) &
                           ~(size_t)255;
    CouplingShape cs{};
    cs.coulomb_k = coulomb_k;
    cs.cutoff = cutoff;
    cs.max_nnp = std::max(n_nnp, 1);
    cs.max_mm = std::max(n_mm, 1);
    cs.chunk = coupling_chunk(cs.max_mm);
    auto f_bytes = [&](int chunk) { return tsz * 3 * (size_t)n_nnp * (size_t)((n_mm + chunk - 1) / chunk); };
    while (e_bytes + f_bytes(cs.chunk) > kCoupleScratchBytes && cs.chunk < 512) cs.chunk += 16;
    if (e_bytes + f_bytes(cs.chunk) > kCoupleScratchBytes)
        return fail(NNP_E_CAPACITY, "coupling partials exceed the static scratch (8 MiB)");
    double* e_part = (double*)scratch;
    void* f_part = (char*)scratch + e_bytes;
    const bool acc = (flags & NNP_FLAG_ACCUMULATE) != 0;
    hipStream_t st = (hipStream_t)stream;
    if (precision == NNP_PREC_FP64)
        e = launch_coupling<double>(cs, n_nnp, (const double*)x_nnp, (const double*)par_nnp, n_mm,
                                    (const double*)x_mm, (const double*)par_mm, out_E, (double*)F_nnp,
                                    (double*)F_mm, e_part, (double*)f_part, acc, st);
    else
        e = launch_coupling<float>(cs, n_nnp, (const float*)x_nnp, (const float*)par_nnp, n_mm,
                                   (const float*)x_mm, (const float*)par_mm, out_E, (float*)F_nnp,
                                   (float*)F_mm, e_part, (float*)f_part, acc, st);
    if (e != hipSuccess) return fail(NNP_E_DEVICE, std::string("coupling launch: ") + hipGetErrorString(e));
    return NNP_OK;
}

}  // extern "C"
