/*
 * nnp.h -- C ABI of the MI355X (gfx950) neural-network-potential library.
 *
 * The library evaluates the NNP term of an NNP/MM simulation: the potential
 * V_NNP(Z, r) of the atoms of the NNP region and the forces F = -grad_r V_NNP
 * (Methods, Eq. 2 and Eq. 3), with positions and forces resident on the GPU
 * (Methods, first optimisation: no CPU<->GPU copies per step).  V_NNP is an
 * ANI-style model: per-atom symmetry-function features (AEVs, the modified
 * Behler-Parrinello functions of ANI with cosine cutoffs, Introduction) fed to
 * one atomic network per element, averaged over an ensemble of networks
 * (Methods, third optimisation: ANI-2x uses 8).  The total charge of Eq. 2 is
 * not an input: the ANI-2x family handles neutral molecules only
 * (Introduction).  One call evaluates one molecule (the low-latency MD case,
 * Methods) or a ragged batch of independent molecules or replicas.
 *
 * Conventions
 *  - Lengths in Angstrom.  Energies in the units of energy_scale times the
 *    network output (627.5094740631 turns Hartree into kcal/mol); forces in
 *    those energy units per Angstrom.
 *  - Coordinates are [n_atoms][3] row-major, forces likewise.
 *  - "device" pointers are HIP device memory of the handle's device (hipMalloc
 *    or torch CUDA tensors); "host" pointers are ordinary memory.
 *  - Every call is asynchronous on the batch's stream unless stated: it returns
 *    after enqueueing, outputs are valid once the stream reaches that point,
 *    and inputs must stay valid until then.
 *  - Errors: every entry point returns an nnp_status.  Invalid arguments are
 *    detected on the host before anything is launched (nothing is written).
 *    Conditions only the device can see (an element index out of range, a
 *    molecule larger than the capacity, a neighbour list overflow) set a
 *    device flag that nnp_get_device_status reads; results of that call are
 *    then unspecified.  nnp_last_error() describes the last host-side error of
 *    the calling thread.  No C++ exception crosses this interface.
 *  - A handle may be used by one host thread and one stream at a time; any
 *    number of handles may coexist.
 */
#ifndef NNP_H
#define NNP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t nnp_status;

#define NNP_OK              0
#define NNP_E_INVALID       1   /* null pointer, size out of range, bad hyper-parameter      */
#define NNP_E_SPECIES       2   /* element (index or atomic number) outside the handle's table:
                                   at creation (bad table) or from the device flag            */
#define NNP_E_CAPACITY      3   /* batch exceeds the capacity given at creation               */
#define NNP_E_NOMEM         4   /* device allocation failed                                   */
#define NNP_E_DEVICE        5   /* a HIP runtime call failed                                  */
#define NNP_E_UNSUPPORTED   6   /* valid request the library does not implement               */

/* Arithmetic of the path. */
#define NNP_PREC_FP64       0   /* everything in FP64 (checking mode)                         */
#define NNP_PREC_FP32       1   /* AEV, networks and forces in FP32; energies summed in FP64  */
#define NNP_PREC_BF16_MLP   2   /* network GEMM operands BF16 with FP32 accumulation; AEV,
                                   activations' epilogues and forces FP32                     */

#define NNP_MAX_SPECIES     8

/* nnp_batch.flags */
#define NNP_FLAG_GRAPH      1u  /* replay a captured HIP graph of the whole evaluation while the
                                   batch shape, every pointer, the flags and the stream stay
                                   the same (first such call runs eagerly and captures); needs
                                   a non-null stream and is ignored while per-kernel timing is
                                   on                                                         */
#define NNP_FLAG_DEVICE_COUNTS 4u /* the batch's molecule and atom counts are read on the device
                                   from nnp_batch.counts (see there); n_mols and n_atoms are
                                   then upper bounds, and a captured graph serves every batch
                                   within the same rounded bounds                             */
#define NNP_FLAG_ACCUMULATE 2u  /* add the results to what the outputs hold instead of
                                   overwriting them (nnp_energy_forces / _f64: out_E and
                                   out_F; nnp_coupling_eval: its energy and both forces), e.g.
                                   to sum V_NNP and the coupling term of Eq. 1 in one buffer  */

/* nnp_model_params.create_flags */
#define NNP_CREATE_TRAINING 1u  /* allocate the training backward's workspace in nnp_create
                                   (FP32 / FP64 handles); without it the first
                                   nnp_energy_forces_backward allocates it                    */

typedef struct nnp_handle nnp_handle;

/*
 * Model description, read once by nnp_create (everything is deep-copied; the
 * caller may free its buffers when nnp_create returns).
 *
 * Featuriser (the published ANI form; the paper names it in the Introduction):
 *   fc(r)  = 0.5 cos(pi r / Rc) + 0.5 for r < Rc, else 0
 *   radial   G_i[n_shf_r*s_j + k] += radial_pref exp(-eta_r (r_ij - shf_r[k])^2) fc(r_ij; rcr)
 *   angular  for each unordered neighbour pair {j,k} of i within rca:
 *            c = cos theta_jik, c' = angle_scale c,
 *            cos(theta' - t_z) = c' cos t_z + sqrt(1 - c'^2) sin t_z, t_z = shf_z[z]
 *            G_i[S*n_shf_r + n_shf_a*n_shf_z*p(s_j,s_k) + n_shf_z*a + z] +=
 *              2 ((1 + cos(theta' - t_z))/2)^zeta
 *                exp(-eta_a ((r_ij + r_ik)/2 - shf_a[a])^2) fc(r_ij; rca) fc(r_ik; rca)
 *            p(b,c), b <= c: row-major index of the upper triangle of S x S.
 *   AEV dimension D = S n_shf_r + S(S+1)/2 n_shf_a n_shf_z (1008 for ANI-2x).
 * Networks: one per (model, element); hidden layers CELU(alpha) (z for z >= 0,
 *   alpha (exp(z/alpha) - 1) otherwise), linear scalar output.  Energy of a
 *   molecule: energy_scale * ( mean over models of the summed atomic outputs
 *   + sum of sae[s_i] ).
 *
 * weights (host, FP64): [model][element][layer] { W (out x in, row-major), b (out) }.
 * This build supports n_shf_r = 16, n_shf_a * n_shf_z = 32, n_layers = 4 with
 * hidden widths that are multiples of 32 (E_UNSUPPORTED otherwise).
 *
 * Element networks of their own sizes (the ANI-2x element networks differ):
 * species_widths [S][n_layers+1] gives element s's widths (first D, last 1,
 * hidden 1..4096, any value); `widths` is then ignored.  The packed weights and
 * parameter gradients follow those widths, so the (model, element) blocks have
 * different lengths.  Internally every element network is zero-padded to the
 * widest one (rounded up to a multiple of 32): zero weights and biases give
 * z = 0, CELU(0) = 0 and no contribution downstream, so the padding changes no
 * result.
 */
typedef struct {
    int32_t n_species;            /* S, 1..NNP_MAX_SPECIES                                */
    int32_t n_shf_r, n_shf_a, n_shf_z;
    double rcr, rca;              /* radial / angular cutoff, rca <= rcr                  */
    double eta_r, eta_a, zeta;
    double angle_scale;           /* 0 < angle_scale < 1 keeps d theta'/d c finite        */
    double radial_pref;
    const double* shf_r;          /* host [n_shf_r] */
    const double* shf_a;          /* host [n_shf_a] */
    const double* shf_z;          /* host [n_shf_z] */

    int32_t n_models;             /* M >= 1 */
    int32_t n_layers;             /* affine layers per network (4) */
    const int32_t* widths;        /* host [n_layers+1]; widths[0] = D, widths[n_layers] = 1 */
    const int32_t* species_widths;/* host [S][n_layers+1] per-element widths, or NULL        */
    double celu_alpha;
    const double* weights;        /* host, FP64, packed as above */
    const double* sae;            /* host [S] or NULL (zeros) */
    double energy_scale;

    int32_t precision;            /* NNP_PREC_* */
    int32_t max_atoms;            /* capacity: atoms per call */
    int32_t max_mols;             /* capacity: molecules per call */
    int32_t max_atoms_per_mol;    /* capacity: atoms of the largest molecule (<= 1024) */
    int32_t device;               /* HIP device ordinal */

    /* Element table (Eq. 2 takes the atomic numbers Z of the NNP atoms):
     * host [S], the atomic number of element s (1..127, all distinct), e.g.
     * {1, 6, 7, 8, 9, 16, 17} for H, C, N, O, F, S, Cl.  With a table, the
     * batches' species arrays hold atomic numbers and an atomic number
     * outside the table raises NNP_E_SPECIES on the device flag; NULL: they
     * hold element indices 0..S-1.  A bad table fails creation with
     * NNP_E_SPECIES. */
    const int32_t* atomic_numbers;
    uint32_t create_flags;        /* 0 or NNP_CREATE_TRAINING */
} nnp_model_params;

/*
 * One evaluation's batch: n_mols molecules in CSR form.  Atoms of molecule b
 * are [mol_offsets[b], mol_offsets[b+1]) of the coordinate/species arrays.
 * Molecules never interact; an empty molecule has zero energy.
 *
 * Device-side counts (NNP_FLAG_DEVICE_COUNTS; the batching of many ragged
 * molecules in one graph-captured launch, Methods, third optimisation): the
 * call reads {n_mols, n_atoms} from the device array `counts` when it runs,
 * and the host fields n_mols and n_atoms are upper bounds of those counts
 * (within the capacities).  The library sizes its launches for the bounds
 * rounded up to powers of two (capped at the capacities), and with
 * NNP_FLAG_GRAPH it keys its captured graph on those rounded bounds instead
 * of the exact sizes: a caller that writes a new batch (coordinates,
 * species, offsets and counts) into the same device buffers replays the same
 * graph, with no re-capture, for every batch within the bounds.  The arrays
 * need hold only the batch itself (mol_offsets [counts[0]+1], atoms
 * [counts[1]]); out_E receives counts[0] energies.  Counts above the rounded
 * bounds, or offsets that do not end at counts[1], set NNP_E_CAPACITY on the
 * device flag.  nnp_aev, nnp_autotune and nnp_energy_forces_backward take
 * host counts only (NNP_E_UNSUPPORTED).
 */
typedef struct {
    int32_t n_mols;               /* 1..max_mols */
    int32_t n_atoms;              /* 0..max_atoms, must equal mol_offsets[n_mols] */
    const int32_t* mol_offsets;   /* device [n_mols+1], non-decreasing, [0] = 0 */
    const int32_t* species;       /* device [n_atoms]: atomic numbers on handles created with an
                                     element table, else element indices 0..S-1 */
    void* stream;                 /* hipStream_t; NULL = the null stream */
    uint32_t flags;               /* NNP_FLAG_GRAPH | NNP_FLAG_ACCUMULATE | NNP_FLAG_DEVICE_COUNTS */
    const int32_t* counts;        /* device [2] {n_mols, n_atoms} with NNP_FLAG_DEVICE_COUNTS, else unused */
} nnp_batch;

/*
 * Create a handle: validate the model, pack its weights for the chosen
 * precision onto the device, and allocate the workspace for the capacities.
 * Device memory is allocated here, with two exceptions: the training
 * backward's workspace (here with NNP_CREATE_TRAINING, else on the first
 * nnp_energy_forces_backward, which can then fail with NNP_E_NOMEM and must
 * not be the first such call under graph capture), and the temporary outputs
 * of nnp_autotune.
 * Returns NNP_OK and *out, or an error (and *out = NULL).
 */
nnp_status nnp_create(const nnp_model_params* params, nnp_handle** out);

/* Release the handle and everything it owns (synchronises its device). */
void nnp_destroy(nnp_handle* h);

/*
 * Energies and forces (Methods, Eq. 2 and Eq. 3), FP32 / BF16-MLP handles.
 *   coords  device float [n_atoms][3]
 *   out_E   device double [n_mols]     (overwritten, or added to with NNP_FLAG_ACCUMULATE)
 *   out_F   device float [n_atoms][3]  (likewise), may be NULL for energies only
 * No allocation; safe to capture in a HIP graph once the batch shape is fixed.
 */
nnp_status nnp_energy_forces(nnp_handle* h, const nnp_batch* b, const float* coords,
                             double* out_E, float* out_F);

/* Same for an NNP_PREC_FP64 handle: coordinates and forces in double. */
nnp_status nnp_energy_forces_f64(nnp_handle* h, const nnp_batch* b, const double* coords,
                                 double* out_E, double* out_F);

/*
 * AEVs of the batch (the featuriser of the path alone), device float or
 * double (FP64 handles) [n_atoms][D], atom order.  For inspection and tests.
 */
nnp_status nnp_aev(nnp_handle* h, const nnp_batch* b, const void* coords, void* out_aev);

/*
 * Training backward of one energies+forces evaluation on the same batch and
 * coordinates: given the loss cotangents grad_E = dL/dE (device double
 * [n_mols], may be NULL = 0) and grad_F = dL/dF (device, coordinate type
 * [n_atoms][3], may be NULL = 0), write
 *   grad_params  device, float (double for FP64 handles), packed exactly like
 *                nnp_model_params.weights: dL/dW for every model and element
 *                (overwritten);
 *   grad_coords  device, coordinate type [n_atoms][3], dL/dx, or NULL:
 *                -gE_b F_i - (H grad_F)_i with H the Hessian of the
 *                molecule's energy in its coordinates (F = -dE/dx, Methods,
 *                Eq. 3); the Hessian-vector product is formed exactly (the
 *                AEV-row tangent through the networks, and the second
 *                derivatives of the featuriser along grad_F).
 */
nnp_status nnp_energy_forces_backward(nnp_handle* h, const nnp_batch* b, const void* coords,
                                      const double* grad_E, const void* grad_F,
                                      void* grad_params, void* grad_coords);

/* Replace the weights (host FP64, packed as in nnp_model_params.weights).
 * Synchronous with respect to the host; the handle must be idle. */
nnp_status nnp_set_weights(nnp_handle* h, const double* weights);

/* Replace the weights from device memory, for training loops that keep their
 * parameters on the GPU (Methods, first optimisation: no CPU<->GPU copies):
 *   params  device [nnp_num_params], packed as nnp_model_params.weights, of
 *           type NNP_PREC_FP64 (double) or NNP_PREC_FP32 (float);
 *   stream  hipStream_t the update is enqueued on (NULL: the null stream).
 * Asynchronous and allocation-free: evaluations enqueued after it on the same
 * stream see the new weights, and captured graphs stay valid (they read the
 * same device buffers).  The values are rounded to the handle's precision
 * exactly as nnp_create rounds host weights, so the result equals a handle
 * created with these weights.  params must stay valid until the stream
 * passes the call; evaluations still running on other streams must finish
 * first. */
nnp_status nnp_set_params(nnp_handle* h, const void* params, int32_t type, void* stream);

/* Number of packed parameters (the length of weights / grad_params). */
int64_t nnp_num_params(const nnp_handle* h);

/* Graph replay bookkeeping of a handle: evaluations captured into a graph
 * and graph replays since creation, and graphs currently cached (each
 * pointer may be NULL). */
nnp_status nnp_graph_stats(const nnp_handle* h, int64_t* captures, int64_t* replays, int32_t* cached);

/* AEV dimension D of the handle's featuriser. */
int32_t nnp_aev_dim(const nnp_handle* h);

/* Read and clear the device-side error flag (synchronises the handle's last
 * stream).  *code is NNP_OK, NNP_E_SPECIES (an element index or atomic number
 * outside the table) or NNP_E_CAPACITY (a molecule above max_atoms_per_mol,
 * rows above the capacity, inconsistent mol_offsets, or an atom with more
 * neighbours within rcr than the list holds: min(max_atoms_per_mol - 1, 192)). */
nnp_status nnp_get_device_status(nnp_handle* h, int32_t* code);

/* Per-kernel timing: when enabled, every kernel launch of the handle is
 * bracketed by HIP events on its stream.  nnp_set_timing (either value)
 * clears the totals.  nnp_kernel_times synchronises with the recorded events
 * and returns, for up to cap kernels, their names (valid until the next call
 * on this thread), launch counts and summed milliseconds since the last
 * nnp_set_timing.  Returns the number of distinct kernels (-1 on a null
 * handle); names/counts/total_ms may be NULL to query the count. */
nnp_status nnp_set_timing(nnp_handle* h, int32_t enable);
/* Restrict the timing above to launches of the kernel called `name` (the
 * names nnp_kernel_times reports, e.g. "mlp_tail"); NULL or "" times every
 * launch again.  Each event record between kernels costs microseconds of GPU
 * time, so timing one kernel perturbs an evaluation least.  Clears the totals
 * like nnp_set_timing; the setting persists across nnp_set_timing calls.
 * NNP_E_INVALID on a null handle. */
nnp_status nnp_set_timing_only(nnp_handle* h, const char* name);
int32_t nnp_kernel_times(nnp_handle* h, int32_t cap, const char** names, int64_t* counts,
                         double* total_ms);

/* ---- tunable variants (the autotuner) -------------------------------------
 * Kernel variants that compute the same quantities (results differ only by
 * floating-point summation order) and differ in speed.  Every knob starts at
 * 0, the built-in automatic choice; nnp_get_knob reports the value in effect.
 *
 *   NNP_KNOB_MLP_PATH     1 = layers 2-3 forward and backward fused in one
 *                             kernel per row tile and model (hidden widths
 *                             256-192-{160..192} only),
 *                         2 = one GEMM per layer and direction.
 *                         auto: 1 when supported, else 2.
 *   NNP_KNOB_GEMM_STAGES  LDS pipeline depth of the layer-1 GEMMs on handles
 *                         with 128-row buckets: 2 or 3 (auto 2: two
 *                         workgroups fit a compute unit); 16-row buckets
 *                         (small batches, FP64) always take 6.
 *   NNP_KNOB_CELL_MIN     molecules with more atoms than this build their
 *                         neighbour lists through cutoff cells, smaller ones
 *                         scan all atoms: 16..1024 (auto 128).
 *   NNP_KNOB_GEMM_WAVES   waves per workgroup of the layer-1 forward GEMM
 *                         of layer-1 path 1 on handles with 128-row buckets:
 *                         4 (2 x 2 waves of 64 x 64) or 8 (2 x 4 waves of
 *                         64 x 32) (auto 8; the backward GEMM always runs 4;
 *                         path 2 always runs 4 waves of 128 x 64).
 *   NNP_KNOB_TAIL_TILE    row tile of the fused layers 2-3 kernel (handles
 *                         with 128-row buckets): 1 = 128 / (operand bytes)
 *                         rows on 4 waves, 2 = half that (at least 16) on 4
 *                         waves, 3 = the full tile on 8 waves (2 x 4); 3 is
 *                         taken as 1 for FP64 (auto 1).
 *   NNP_KNOB_L1_PATH      layer-1 GEMMs of BF16 handles with 128-row
 *                         buckets: 1 = both operands staged through LDS
 *                         (the GEMM_STAGES / GEMM_WAVES knobs apply),
 *                         2 = activation rows through LDS and the weights
 *                         loaded into registers from a fragment-ordered copy
 *                         (128 x 256 tiles; needs M*H1 and the padded AEV
 *                         length to be multiples of 256).  auto: 2 when
 *                         supported, else 1.
 *   NNP_KNOB_ATOM_CHUNK   central atoms per workgroup of the featuriser and
 *                         force kernels (4 waves): 4, 8 or 16.  Fewer atoms
 *                         per workgroup spread a small batch over more
 *                         compute units; more share the staging of their
 *                         molecule.  auto: 16 when the capacity gives at
 *                         least 1024 workgroups at 16, else 4.
 *   NNP_KNOB_FORCE_SUM    1 = forces summed with floating-point atomic adds
 *                         (the last bits vary from run to run), 2 = every
 *                         contribution rounded to a 64-bit fixed-point
 *                         integer (units of 2^-32) and summed with integer
 *                         adds, converted to the force type once: bitwise
 *                         identical forces on every run, stream and launch
 *                         shape (the rest of an evaluation already is).
 *                         auto: 1.  The autotuner leaves this knob alone.
 *   NNP_KNOB_FORCE_PATH   force kernel: 1 = each atom's dE/dAEV row staged in
 *                         LDS, 2 = read from global memory (cache hits),
 *                         leaving the LDS to the force sums.  auto: 2.
 *   NNP_KNOB_PIPELINE     1 = one evaluation on the batch's stream; 2 = the
 *                         molecules split in two halves evaluated on two
 *                         streams (the handle's own second stream, forked from
 *                         and joined back into the batch's), so that one half's
 *                         featuriser and force kernels run beside the other
 *                         half's network kernels.  Needs a second set of row
 *                         buffers, allocated when the knob is first set to 2
 *                         (by nnp_set_knob or the autotuner).  Batches of one
 *                         molecule, device counts and nnp_aev run as one part.
 *                         auto: 1 (each kernel of one part already fills the
 *                         chip; the overlap has measured slower).
 *
 * Setting a knob drops the handle's captured graphs.  Invalid knob ids or
 * values return NNP_E_INVALID (a fused path on unsupported widths returns
 * NNP_E_UNSUPPORTED). */
enum {
    NNP_KNOB_MLP_PATH = 0,
    NNP_KNOB_GEMM_STAGES = 1,
    NNP_KNOB_CELL_MIN = 2,
    NNP_KNOB_TAIL_TILE = 3,
    NNP_KNOB_GEMM_WAVES = 4,
    NNP_KNOB_ATOM_CHUNK = 5,
    NNP_KNOB_L1_PATH = 6,
    NNP_KNOB_FORCE_SUM = 7,
    NNP_KNOB_FORCE_PATH = 8,
    NNP_KNOB_PIPELINE = 9,
    NNP_N_KNOBS = 10
};
nnp_status nnp_set_knob(nnp_handle* h, int32_t knob, int32_t value);
nnp_status nnp_get_knob(nnp_handle* h, int32_t knob, int32_t* value);

/* Autotuner: times the candidates of every knob on this batch (one warm-up
 * and `reps` evaluations each, HIP events on the batch's stream), knob by
 * knob, and keeps the fastest on the handle.  coords are float (double for
 * FP64 handles).  If cache_path is non-NULL the choice is looked up first in
 * that file (JSON lines, one object per key: device architecture, precision,
 * model shape and capacity) and, when tuned afresh, appended to it.  If
 * report is non-NULL a JSON object with the key, the chosen values and the
 * timings of every candidate (microseconds per evaluation) is written into it
 * (truncated to report_cap bytes).  Allocates temporary outputs; synchronises
 * the stream; not for use under graph capture. */
nnp_status nnp_autotune(nnp_handle* h, const nnp_batch* b, const void* coords, int32_t reps,
                        const char* cache_path, char* report, int32_t report_cap);

/* ---- NNP-MM coupling (mechanical embedding) --------------------------------
 * The coupling term of an NNP/MM energy (Methods, Eq. 4): every NNP atom i
 * interacts with every MM atom j through
 *
 *   k q_i q_j / r_ij + 4 eps_ij ((sigma_ij / r_ij)^12 - (sigma_ij / r_ij)^6),
 *
 * k = 1 / (4 pi eps0) in the caller's units (332.0637133 kcal/mol A / e^2 for
 * kcal/mol, A, e), with Lorentz-Berthelot pair parameters sigma_ij =
 * (sigma_i + sigma_j) / 2 and eps_ij = sqrt(eps_i eps_j).  cutoff > 0 drops
 * every pair with r_ij >= cutoff (a plain truncation); cutoff = 0 keeps all.
 *
 * nnp_coupling_create: precision NNP_PREC_FP64 or NNP_PREC_FP32 (the operand
 * and force type; the energy is always summed in FP64); capacities max_nnp
 * (1..1024) and max_mm (1..2^22); allocates its workspace on `device`.
 *
 * nnp_coupling_eval: all arrays are device pointers of the handle's type:
 * x_nnp [n_nnp][3], par_nnp [n_nnp][3] = (q, sigma, eps), likewise for MM;
 * out_E one double; F_nnp [n_nnp][3] and F_mm [n_mm][3] receive -dV/dx.
 * flags: 0 overwrites the outputs, NNP_FLAG_ACCUMULATE adds to them (for
 * example onto the NNP energy and forces of the same step).  Runs on
 * `stream` (a hipStream_t); allocates nothing; the result is independent of
 * launch configuration and bitwise repeatable (no atomics).  Sizes above the
 * capacities return NNP_E_CAPACITY; null pointers NNP_E_INVALID (n = 0 sides
 * may pass NULL arrays). */
typedef struct nnp_coupling nnp_coupling;
nnp_status nnp_coupling_create(int32_t precision, int32_t max_nnp, int32_t max_mm, double coulomb_k,
                               double cutoff, int32_t device, nnp_coupling** out);
void nnp_coupling_destroy(nnp_coupling* c);
nnp_status nnp_coupling_eval(nnp_coupling* c, int32_t n_nnp, const void* x_nnp, const void* par_nnp,
                             int32_t n_mm, const void* x_mm, const void* par_mm, double* out_E,
                             void* F_nnp, void* F_mm, void* stream, uint32_t flags);

/*
 * nnp_coupling_eval without a handle and without any allocation, for callers
 * that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  Same arguments, result
 * and flags as nnp_coupling_eval on a handle of this precision, coulomb_k and
 * cutoff; runs on the current HIP device.
 *
 * Its partial sums live in a static device array of 8 MiB that the library
 * holds on every GPU it runs on until the process ends: ceil(n_mm / 64)
 * doubles plus 3 n_nnp ceil(n_mm / chunk) values of the operand type, where
 * chunk is the handle's MM-atoms-per-wave rule widened (up to 512) until they
 * fit.  The 64-atom ligand in 47,648 MM atoms needs 2.3 MB (FP32) or 4.6 MB
 * (FP64).  Larger systems, or n_nnp > 1024 or n_mm > 2^22, return
 * NNP_E_CAPACITY before anything is launched.  The first call on a device
 * looks up that device's copy of the array (no allocation).
 *
 * Every call on one GPU shares that array: calls that overlap in time on one
 * GPU (two streams, two host threads) race and give wrong results; serialise
 * them.  Nothing in the array needs clearing: every partial a call reads is
 * written earlier in the same call.
 */
nnp_status nnp_coupling_eval_noalloc(int32_t precision, double coulomb_k, double cutoff, int32_t n_nnp,
                                     const void* x_nnp, const void* par_nnp, int32_t n_mm,
                                     const void* x_mm, const void* par_mm, double* out_E, void* F_nnp,
                                     void* F_mm, void* stream, uint32_t flags);

/* Message of the calling thread's last host-side error ("" if none). */
const char* nnp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* NNP_H */
