/*
 * dp.h -- C ABI of the MI355X (gfx950) deep-potential energy/force/virial library.
 *
 * The operation: for one configuration of atoms (the atom group an MD engine
 * hands to the potential each step -- positions, types, periodic box; paper,
 * Section III), evaluate the attention-based deep potential (Section II: a
 * type-embedded per-neighbour embedding net, self-attention layers that update
 * that representation residually, a fitting net giving each atom's energy,
 * E = sum of atomic energies) and its forces F = -dE/dx (Section II) and
 * virial, using neighbour lists within the model cutoff over periodic
 * boundaries (Sections I, II, IV).
 *
 * Conventions
 *   Units: Angstrom, eV, eV/Angstrom.  coords are [natoms][3] row-major float64;
 *   types are int32 in [0, ntypes); box is 3 row vectors [3][3] float64 and must
 *   be orthorhombic with every edge >= 2 * rc, or NULL for open boundaries.
 *   forces [natoms][3] float64; virial [3][3] row-major float64,
 *   Xi_ab = -sum_i sum_{j in N(i)} Delta_ij,a dE/dDelta_ij,b (Delta_ij = x_j - x_i, minimum image).
 *   atom_energy [natoms] float64, may be NULL.
 * Ownership
 *   The caller owns every input and output buffer; calls borrow them for their
 *   duration only.  A dp_model owns its device weights and a grow-only device
 *   workspace: after the first call at a given natoms no further device
 *   allocation happens for natoms <= that size.  A dp_model is not thread-safe.
 * Errors
 *   Every int-returning call returns DP_OK (0), a positive warning (outputs
 *   valid but flagged) or a negative error (outputs untouched).  dp_last_error()
 *   gives a thread-local human-readable detail of the last failure.
 */
#ifndef DP_MI355X_H
#define DP_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dp_model dp_model;
typedef struct dp_server dp_server;

/* Arithmetic of the dense products (embedding, attention, fitting).  DP_FP32:
 * float32 operands, float32 accumulation.  DP_BF16: bfloat16 operands (round to
 * nearest even) with float32 accumulation; environment, softmax, LayerNorm,
 * tanh, descriptor contraction and force assembly stay float32 in both. */
enum { DP_FP32 = 0, DP_BF16 = 1 };

enum {
  DP_OK = 0,
  DP_WARN_SEL_OVERFLOW = 1, /* some atom had more than sel neighbours; the sel
                               nearest (ties by index) were kept               */
  DP_ERR_ARG = -1,          /* NULL pointer, natoms < 1, bad precision/device  */
  DP_ERR_MODEL_FILE = -2,   /* unreadable or malformed model file             */
  DP_ERR_TYPE = -3,         /* an atom type outside [0, ntypes)               */
  DP_ERR_BOX = -4,          /* non-orthorhombic box or an edge < 2 rc         */
  DP_ERR_OVERLAP = -5,      /* two atoms at distance 0                        */
  DP_ERR_NONFINITE = -6,    /* NaN or infinite coordinate or box              */
  DP_ERR_OOM = -7,          /* device allocation failed                       */
  DP_ERR_TOO_LARGE = -8,    /* natoms beyond the library limit, or more than
                               DP_MAX_CANDIDATES atoms within rc of one atom  */
  DP_ERR_HIP = -9,          /* a HIP runtime call failed                      */
  DP_ERR_TIMEOUT = -10
};

#define DP_MAX_CANDIDATES 512

/* Load a model file (format: 128-byte header 'DPAMDv01' + float64 arrays) onto
 * HIP device `device`, converting the weights to `precision` (DP_FP32 or
 * DP_BF16).  On success *out owns the model; free it with dp_model_free. */
int dp_model_load(const char *path, int precision, int device, dp_model **out);
void dp_model_free(dp_model *m);

/* Host-only check of a model file; makes no HIP call, so it runs without a GPU.
 * Reads the file, builds the weight image dp_model_load would upload for
 * `precision`, points the kernels' weight structures into it and checks that
 * every pointer the kernels of that precision read is set and lies inside the
 * image (DP_ERR_MODEL_FILE naming the member otherwise).  unbind, when not NULL,
 * names one member to clear before the check (a self-test of the check itself).
 * *image_bytes (may be NULL) receives the size of the device weight image. */
int dp_check_model_file(const char *path, int precision, const char *unbind, size_t *image_bytes);

/* Cutoff rc (Angstrom), neighbour capacity sel, number of atom types. Any
 * output pointer may be NULL. */
int dp_model_info(const dp_model *m, double *rc, int *sel, int *ntypes);

/* Energy, forces and virial of one configuration; host buffers, synchronous.
 * energy: 1 double; forces: [natoms][3]; virial: [3][3]; atom_energy: [natoms]
 * or NULL.  forces and virial may be NULL to skip the backward pass. */
int dp_compute(dp_model *m, int64_t natoms, const double *coords, const int32_t *types,
               const double *box, double *energy, double *forces, double *virial,
               double *atom_energy);

/* Same on device buffers, enqueued on the HIP stream `hip_stream` (NULL = the
 * null stream).  box_host is a host pointer (or NULL).  d_energy: 1 double,
 * d_forces [natoms][3], d_virial [9], d_atom_energy [natoms] (or NULL); d_forces
 * and d_virial may both be NULL to run the energy pass only (see
 * dp_backward_device).  Inputs are validated on the device; the call waits for
 * the stream once at the end to read the status word, so results are ready on
 * return. */
int dp_compute_device(dp_model *m, int64_t natoms, const double *d_coords, const int32_t *d_types,
                      const double *box_host, double *d_energy, double *d_forces, double *d_virial,
                      double *d_atom_energy, void *hip_stream);

/* After an energy-only dp_compute_device on this model (and no other call in
 * between), run the hand-written backward pass: d_grad_coords[natoms][3] =
 * grad_energy * dE/dx, where grad_energy is one double on the device.
 * d_virial (9 doubles, or NULL) receives the virial scaled by grad_energy. */
int dp_backward_device(dp_model *m, const double *d_grad_energy, double *d_grad_coords,
                       double *d_virial, void *hip_stream);

/* Neighbour lists as the library builds them: nlist [natoms][sel] int32 sorted
 * ascending per atom and padded with -1, nnei [natoms], *overflow = number of
 * atoms whose list was truncated to sel.  Host buffers, synchronous. */
int dp_debug_neighbors(dp_model *m, int64_t natoms, const double *coords, const double *box,
                       int32_t *nlist, int32_t *nnei, int64_t *overflow);

/* Pair gradients of the last step that ran the backward pass on this model:
 * g[natoms][sel][4] float32, g[i][s] = dE_i/dDelta_ij for j = nlist[i][s]
 * (x, y, z, 0; padded slots zero).  Host buffer, synchronous.  For diagnostics. */
int dp_debug_pair_grads(dp_model *m, int64_t natoms, float *g);

/* Per-phase device timing with HIP events recorded on each call's stream.
 * enable != 0 clears and starts accumulating, 0 stops.  dp_profile_read fills,
 * for up to `max` phases, the summed milliseconds and the number of calls:
 * phase 0 neighbour lists, 1 descriptor forward, 2 fitting net, 3 energy
 * reduction (energy-only calls; a full step reduces the energy with the virial in
 * phase 5), 4 descriptor backward, 5 forces, energy and virial reductions.  Returns the number
 * of phases (DP_NPHASES). */
#define DP_NPHASES 6
int dp_profile_enable(dp_model *m, int enable);
int dp_profile_read(const dp_model *m, double *ms, int64_t *calls, int max);

/* One GPU's share of a spatially decomposed system (paper, Section III: the DP
 * group is spread over ranks, each holding its atoms plus a ghost region; the
 * ghost forces have to be returned to the owners).  The first n_owned atoms of
 * d_coords/d_types are this GPU's own atoms, the rest (natoms - n_owned) its
 * ghosts: copies of atoms owned elsewhere that lie within rc of an owned atom, in
 * the same frame (box_host periodic, or NULL with unwrapped coordinates).  E_i and
 * the pair gradients g_ij = dE_i/dDelta_ij are computed for owned i only, with
 * neighbours among all natoms.  Outputs (device):
 *   d_energy[0]  = sum of E_i over the owned atoms;
 *   d_forces[natoms][3] = sum_{owned i} of the terms this share contributes:
 *       row k gets  sum_j g_kj (k owned)  -  sum_{owned i: k in N(i)} g_ik,
 *     so owned rows hold their forces minus what other shares' centres add, and
 *     ghost rows hold the contributions to be returned to the owners;
 *   d_virial[9]  = -sum_{owned i} sum_j Delta_ij (x) g_ij;
 *   d_atom_energy[n_owned] (or NULL) = E_i of the owned atoms.
 * Adding every share's d_forces rows into the owners' atoms, and summing the
 * energies and virials, gives the whole system's E, F and virial.  n_owned =
 * natoms is dp_compute_device.  Synchronous on hip_stream; fresh neighbour lists
 * (dp_set_skin and dp_set_graph do not apply). */
int dp_compute_owned_device(dp_model *m, int64_t natoms, int64_t n_owned, const double *d_coords,
                            const int32_t *d_types, const double *box_host, double *d_energy, double *d_forces,
                            double *d_virial, double *d_atom_energy, void *hip_stream);

/* Allocation-free variant of dp_compute_device, for callers that cannot allocate
 * device memory during a step: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc.  Same arguments, results and errors as
 * dp_compute_device (fresh neighbour lists each call; dp_set_skin and
 * dp_set_graph do not apply), bitwise the same results.  The workspace is a
 * static device array of 128 MiB per GPU, reserved when the library's code is
 * loaded on that GPU and held until the process ends; it fits natoms <=
 * DP_NOALLOC_MAX_ATOMS, and larger systems get DP_ERR_TOO_LARGE.  The call makes
 * no device or host allocation (dp_model_load sets up the array's address, pinned
 * staging and streams once per device).  Every call on a GPU shares that GPU's
 * array: calls that overlap in time on one GPU (from several threads, streams or
 * models) race and must be serialised by the caller.  The array keeps the last
 * call's contents; the step clears what it needs cleared itself. */
#define DP_NOALLOC_MAX_ATOMS 1024
int dp_compute_device_noalloc(dp_model *m, int64_t natoms, const double *d_coords, const int32_t *d_types,
                              const double *box_host, double *d_energy, double *d_forces,
                              double *d_virial, double *d_atom_energy, void *hip_stream);

/* Several independent periodic systems in one step (paper, Section III: the
 * engine hands the potential one atom group per step; a server batches many).
 * System k has natoms[k] atoms, stored consecutively in d_coords [sum][3] and
 * d_types [sum], and the periodic box boxes[9k .. 9k+8] (host array; every box
 * orthorhombic with edges >= 2 rc -- open boundaries are not accepted here).
 * Outputs on the device: d_energy [nsys], d_forces [sum][3] (or NULL),
 * d_virial [nsys][9] (or NULL).  Each system's results are those of a
 * dp_compute_device call on it alone.  Enqueued on hip_stream; waits for it at
 * the end.  The batch's lists may not need more than 64^3 cells in total. */
int dp_compute_batch_device(dp_model *m, int nsys, const int64_t *natoms, const double *boxes,
                            const double *d_coords, const int32_t *d_types, double *d_energy,
                            double *d_forces, double *d_virial, void *hip_stream);

/* Several fitting heads on one descriptor (paper, Section II: the multi-task
 * pre-trained models share one descriptor between output branches, e.g. the
 * solvated-protein and small-molecule branches of Section IV).  A model file may
 * carry up to 4 fitting nets; every step evaluates the descriptor once and all
 * heads on it, and reports the weighted combination E = sum_h w_h E^h as its
 * energy, with forces and virial of that combination (one backward pass through
 * the shared descriptor).  The weights start as (1, 0, ...): head 0 alone, the
 * single-head result bit for bit.
 *   dp_model_heads:      *nheads = the number of fitting heads (1 .. 4).
 *   dp_set_head_weights: w[nheads] (finite; DP_ERR_ARG if nheads differs from the
 *                        model's); a weight of 0 skips that head's backward.
 *                        Applies to every later call, graphs included.
 *   dp_head_energies:    each head's own energy E^h of the last step, for its
 *                        first nsys systems: energies[nsys][nheads] (host,
 *                        synchronous); models with several heads only. */
int dp_model_heads(const dp_model *m, int *nheads);
int dp_set_head_weights(dp_model *m, int nheads, const double *weights);
int dp_head_energies(dp_model *m, int nsys, double *energies);

/* Neighbour-list reuse across calls (paper, Section IV: Verlet lists with a
 * buffer, rebuilt every 10 steps).  With skin > 0 a list within rc + skin
 * (at most 192 entries per atom) is built on the first call and then every
 * rebuild_every calls with the same natoms and box; every call in between
 * filters it to rc at the current coordinates.  The filtered lists equal a fresh
 * search bit for bit: each call checks on the device that no atom moved by half
 * the skin since the build (and that no skin row was full), and if one did the
 * call is redone with a fresh build.  Boxes with an edge < 2 (rc + skin) use a
 * fresh search every call.  skin = 0 switches reuse off.  dp_skin_stats: skin
 * lists built so far and, of those, the builds forced by the check. */
int dp_set_skin(dp_model *m, double skin, int rebuild_every);
int dp_skin_stats(const dp_model *m, int64_t *builds, int64_t *forced);

/* chunk_atoms > 0: dp_compute_device (fresh lists, eager) evaluates the centre
 * atoms of a larger system in chunks of chunk_atoms: every chunk builds the
 * lists and runs the descriptor, fitting and backward for its own atoms, the last
 * one then gathers the forces and reduces energy and virial.  Same results, bit
 * for bit; the continuous-batching server splits large requests the same way so
 * that small requests can run between the chunks.  0 switches chunking off. */
int dp_set_chunk(dp_model *m, int64_t chunk_atoms);

/* enable != 0: dp_compute_device captures its step (every kernel launch and
 * the small host-to-device copies of the cell grid) into a HIP graph the first
 * time it sees a configuration (natoms, buffer pointers, box, stream, list mode)
 * and replays the graph on later calls with the same configuration; up to 4
 * configurations are kept.  The graph reads the coordinates at replay time.
 * Per-phase profiling (dp_profile_enable) runs the eager path instead.  With
 * hip_stream NULL a graph runs on a stream of the model's own, ordered after the
 * work already queued on the null stream. */
int dp_set_graph(dp_model *m, int enable);

/* Continuous-batching server over one model (the model must not be used
 * otherwise while the server exists; the serving extension of the paper's setting,
 * Section III, where the engine hands the potential one system per step).
 * Requests are periodic systems; each is copied on submit and queued.  Up to
 * max_inflight (1..8) work items run at once, each on its own stream:
 *   - requests of at most 8192 atoms are packed, in arrival order, into batched
 *     steps of at most 8192 atoms (dp_compute_batch_device semantics);
 *   - a larger request is split into chunks of 8192 centre atoms (dp_set_chunk
 *     semantics) on a workspace of its own; after each chunk it goes to the back
 *     of the queue, so requests that arrived meanwhile run first.
 * Admission by device memory: the max_inflight batch workspaces (8192 atoms
 * each, dp_server_footprint bytes per atom) plus the workspaces of the large
 * requests in progress stay within hbm_budget_bytes; dp_server_create refuses a
 * budget below max_inflight batches, and dp_submit refuses (DP_ERR_TOO_LARGE) a
 * system that could never fit.  dp_submit validates the request (types, finite
 * coordinates, box) and never waits for the GPU.  dp_wait blocks up to
 * timeout_s seconds (< 0: no limit; DP_ERR_TIMEOUT on expiry, the request stays
 * pending), copies energy (1), forces ([natoms][3]) and virial (9) to host
 * buffers (any may be NULL), gives the latency from submit to completion, and
 * releases the request.  A request whose batch fails is re-run alone so that its
 * own status is reported.  Results equal dp_compute on the request alone, bit
 * for bit.  dp_server_stats: nearest-rank p50/p99 latency over completed
 * requests, atoms completed per second from the first submit to the last
 * completion, completed requests, work items launched, largest item in atoms
 * (any output may be NULL).  dp_submit/dp_wait/dp_server_stats may be called
 * from any thread; dp_server_free waits for queued work to finish. */
size_t dp_server_footprint(const dp_model *m, int64_t natoms);
int dp_server_create(dp_model *m, size_t hbm_budget_bytes, int max_inflight, dp_server **out);
int dp_submit(dp_server *s, int64_t natoms, const double *coords, const int32_t *types,
              const double *box, uint64_t *request_id);
int dp_wait(dp_server *s, uint64_t request_id, double timeout_s, double *energy, double *forces,
            double *virial, double *latency_s);
int dp_server_stats(dp_server *s, double *p50_s, double *p99_s, double *atom_evals_per_s,
                    int64_t *completed, int64_t *batches, int64_t *max_batch_atoms);
void dp_server_free(dp_server *s);

/* Velocity-Verlet NVE on the device with this model's forces (paper, Section IV:
 * MD with a fixed time step; a test harness for energy conservation, not part
 * of the timed step).  d_coords [natoms][3] (Angstrom) and d_vel [natoms][3]
 * (Angstrom/fs) are device float64 arrays advanced in place by nsteps steps of
 * dt_fs; masses[ntypes] in amu (host).  epot and ekin (host, nsteps + 1 doubles
 * each, or NULL) receive the potential and kinetic energy (eV) before the first
 * step and after each step.  Uses dp_compute_device for every force call, so
 * dp_set_skin and dp_set_graph apply.  Returns the worst status of the steps. */
int dp_nve_run(dp_model *m, int64_t natoms, double *d_coords, double *d_vel, const int32_t *d_types,
               const double *masses, const double *box, double dt_fs, int nsteps, double *epot, double *ekin,
               void *hip_stream);

/* ---------------------------------------------------------------------------
 * GNN-variant model (paper, Section II: the message-passing descriptor over
 * bonds and angles of its second model family, in place of attention).
 * Model: edges (i, j) within rc; angles at i are the ordered pairs (p, q), p != q,
 * of the first asel neighbours of i (list order) closer than rca; node (64), edge
 * (64) and angle (32) features, three layers each updating angles, then edges (with
 * the switched angle messages), then nodes (with the switched mean of their edges);
 * a fitting net 64 -> 128 -> 128 -> 1 on the final node features; E = sum E_i.
 * Every term an edge or angle adds carries a switch that vanishes at its cutoff.
 * The model file (magic DPGNNv01: a 128-byte header of sizes, rc, rcs, rca, then the
 * float64 arrays) fixes node/edge/angle widths 64/64/32, three layers, fitting
 * width 128, sel = 120, asel <= 48 and ntypes = 5.
 *
 * dp_gnn_load: precision DP_FP32 or DP_BF16 (operands of every feature-by-weight
 *   product; features are stored and combined in float32 either way).
 * dp_gnn_compute_device: arguments, units and outputs as dp_compute_device (device
 *   pointers, box on the host or NULL, energy required, the rest may be NULL).  The
 *   neighbour lists must be complete: an atom with more than sel neighbours within
 *   rc gives DP_ERR_TOO_LARGE (outputs untouched).  The call sizes its angle buffers
 *   from the step's angle count (one host round trip) and returns after the step
 *   has finished on the stream.  A dp_gnn owns grow-only device buffers of about
 *   190 KB per atom and 512 bytes per angle; it is not thread-safe.
 * dp_gnn_info: rc, rca, sel, asel of the model (pointers may be NULL).
 * dp_gnn_graph_size: edges (sum of the list lengths), angle-list edges (sum of nc
 *   over the atoms that have angles) and angles of the last successful step
 *   (pointers may be NULL).
 * dp_gnn_profile_enable / dp_gnn_profile_read: per-phase device time from HIP events
 *   on the step's stream, accumulated over calls since enabling (which clears it):
 *   phase 0 lists (cell list, neighbour lists, angle offsets), 1 the three forward
 *   layers with the fitting net, 2 the three backward layers, 3 forces and reductions.
 *   read fills ms[k], calls[k] for k < min(max, 4) and returns that count. */
typedef struct dp_gnn dp_gnn;
int dp_gnn_load(const char *path, int precision, int device, dp_gnn **out);
void dp_gnn_free(dp_gnn *m);
int dp_gnn_info(const dp_gnn *m, double *rc, double *rca, int *sel, int *asel);
int dp_gnn_compute_device(dp_gnn *m, int64_t natoms, const double *d_coords, const int32_t *d_types,
                          const double *box_host, double *d_energy, double *d_forces, double *d_virial,
                          double *d_atom_energy, void *hip_stream);
int dp_gnn_graph_size(const dp_gnn *m, int64_t *edges, int64_t *angle_edges, int64_t *angles);
int dp_gnn_profile_enable(dp_gnn *m, int enable);
int dp_gnn_profile_read(const dp_gnn *m, double *ms, int64_t *calls, int max);

/* ---------------------------------------------------------------------------
 * Repformer-style model (paper, Section II: the DPA2 family, whose layers update a
 * single-atom and a pair representation and pass messages from neighbour to
 * neighbour, so the receptive field grows by rc per layer).
 * Model: node features g1 (64) per atom and pair features g2 (32) per edge (j in
 * the rc list of i); three layers, each: the pair update from the neighbour's g1,
 * a switch-gated self-attention over i's pair features (one head, width 32,
 * weights sw_k exp(Q_j.K_k / sqrt 32) normalised, times rhat_j.rhat_k), and the
 * node update from the contraction T T[:4]^T (T = sum_j g2_ij R_ij^T / sel) and
 * the convolution sum_j sw_ij g2_ij * g1_j[:32] / sel; fitting 64 -> 128 -> 128
 * -> 1 on g1; E = sum E_i.  Model file: magic DPREPv01 (128-byte header of sizes,
 * rc, rcs, then the float64 arrays); node/pair widths 64/32, 4 axis columns,
 * three layers, fitting width 128, sel = 120, ntypes = 5.  Float32 arithmetic.
 *
 * dp_rep_compute_device: arguments, units and outputs as dp_compute_device.  Lists
 *   must be complete (more than sel neighbours within rc: DP_ERR_TOO_LARGE).
 *   Returns after the step has finished on the stream.  A dp_rep owns grow-only
 *   device buffers of about 120 KB per atom; it is not thread-safe.
 * dp_rep_edges: edges (sum of the list lengths) of the last successful step.
 * dp_rep_profile_enable / dp_rep_profile_read: per-phase device time as for the GNN
 *   model (0 lists, 1 forward layers with the fitting net, 2 backward layers, 3
 *   forces and reductions). */
typedef struct dp_rep dp_rep;
int dp_rep_load(const char *path, int device, dp_rep **out);
void dp_rep_free(dp_rep *m);
int dp_rep_compute_device(dp_rep *m, int64_t natoms, const double *d_coords, const int32_t *d_types,
                          const double *box_host, double *d_energy, double *d_forces, double *d_virial,
                          double *d_atom_energy, void *hip_stream);
int dp_rep_edges(const dp_rep *m, int64_t *edges);
int dp_rep_profile_enable(dp_rep *m, int enable);
int dp_rep_profile_read(const dp_rep *m, double *ms, int64_t *calls, int max);

/* Static description of a status code; never NULL. */
const char *dp_status_string(int status);
/* Thread-local detail of the last failure in this thread ("" if none). */
const char *dp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DP_MI355X_H */
