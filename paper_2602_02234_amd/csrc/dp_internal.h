// Host/device structures shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>

#include "dp_common.h"

namespace dp {

// Cell grid over the box (periodic) or over the atoms' bounding box (open).
struct Grid {
  double origin[3];
  double L[3];      // periodic box edges, or bounding-box extent
  double invL[3];   // 1 / L (periodic minimum image)
  double cw[3];     // cell edge, >= rc (1 + 1e-9) unless there is a single cell
  double icw[3];    // 1 / cw
  int nc[3];
  int periodic;
  int ncells;
  int cell_base;    // first cell of this system in a multi-system cell array
  int pad_;
};

constexpr int MAX_CELLS_PER_DIM = 64;
constexpr int MAX_CELLS = MAX_CELLS_PER_DIM * MAX_CELLS_PER_DIM * MAX_CELLS_PER_DIM;
constexpr int CAND_CAP = 512;  // neighbours within rc one atom may have before DP_ERR_TOO_LARGE
constexpr int SKIN_CAP = 192;  // entries per row of the skin list (within rc + skin)

// Status bits written by kernels into the workspace flag word.  STALE: an atom moved by
// half the skin since the skin list was built; SKIN_FULL: a skin row overflowed.  Both
// make the host redo the step with a fresh search.  INCOMPLETE: set only for the
// message-passing models, which refuse truncated lists.
enum : unsigned {
  FLAG_OVERLAP = 1u, FLAG_TYPE = 2u, FLAG_NONFINITE = 4u, FLAG_TOO_DENSE = 8u, FLAG_STALE = 16u,
  FLAG_SKIN_FULL = 32u,
  FLAG_INCOMPLETE = 64u,  // a list was truncated to sel and the model needs complete lists
  FLAG_ERRORS = 127u,     // any of the above: outputs are not written
};

constexpr int MAXH = 4;  // fitting heads one model may carry

// Device weight tables read by both precision paths: biases, the first embedding
// layer (its type part folded into Bt), LayerNorm parameters and, per fitting head, the
// fitting biases and last layer.
struct Tables {
  const float *w1s;   // [E1]            first embedding layer, s column
  const float *Bt;    // [NTYPES][NTYPES][E1]  type part + bias of the first layer
  const float *b2;    // [E2]
  const float *b3;    // [M]
  const float *gamma[NATTN];
  const float *beta[NATTN];
  int nheads;         // fitting heads (1 .. MAXH)
  double hw[MAXH];    // head weights: E_i = sum_h hw[h] E_i^h (forces and virial follow)
  const float *c1[MAXH], *c2[MAXH], *c3[MAXH];
  const float *F4[MAXH];    // [FH]  last layer, float32 copy for the backward
  // The last layer's energy terms stay float64: E_i = y3 . F4 + c4 + ebias[t_i] is summed
  // in float64 from float32 y3, so the large, shared F4 and c4 add no rounding of their own.
  const double *F4d[MAXH];  // [FH]
  double c4[MAXH];
  const double *ebias[MAXH];  // [NTYPES]
};

// GEMM operands of the float32 path, T = float, row-major as named.
template <typename T> struct Weights : Tables {
  const T *W2T;       // [E2][E1]
  const T *W2;        // [E1][E2]
  const T *W3T;       // [M][E2]
  const T *W3;        // [E2][M]
  const T *WqkT[NATTN];  // [M][M]  (WQ WK^T / sqrt(d))^T
  const T *Wqk[NATTN];   // [M][M]
  const T *WvoT[NATTN];  // [M][M]  (WV WO)^T
  const T *Wvo[NATTN];   // [M][M]
  const T *F1T[MAXH];    // [FH][ND]  per fitting head
  const T *F1[MAXH];     // [ND][FH]
  const T *F2T[MAXH];    // [FH][FH]
  const T *F2[MAXH];
  const T *F3T[MAXH];
  const T *F3[MAXH];
};

// Extra device weights of the bfloat16 path: GEMM operands zero-padded to MFMA
// tile multiples and stored [output column][k] (k contiguous, 16-byte rows), so
// every MFMA fragment is one 16-byte load.  Feature width 100 is padded to 112,
// embedding widths 25/50 to 32/64, the fitting width 240 to 256 along k.  The
// fitting operands come as a two-term split w = hi + lo (both bf16).
struct WeightsB16 {
  const bf16_t *W2T;           // [64][32]    W2T[c][k] = W2[k][c]
  const bf16_t *W3T;           // [112][64]   W3T[m][k] = W3[k][m]
  const bf16_t *W3;            // [64][112]   W3[c][m]
  const bf16_t *W2;            // [32][64]    W2[e1][e2]
  // attention weights, [112][112] each, in MFMA fragment order (see mm_g)
  const bf16_t *WqkT[NATTN];   // WqkT[c][k] = Wqk[k][c]
  const bf16_t *Wqk[NATTN];
  const bf16_t *WvoT[NATTN];
  const bf16_t *Wvo[NATTN];
  // fitting operands per head, hi and lo parts, in MFMA fragment order (fragment (t, s)
  // of a [cols][K] matrix at ((t * K / 32 + s) * 64 + lane) * 8)
  const bf16_t *F1T[MAXH][2];  // [240][1600]
  const bf16_t *F1[MAXH][2];   // [1600][256]
  const bf16_t *F2T[MAXH][2];  // [240][256]
  const bf16_t *F2[MAXH][2];   // [240][256]
  const bf16_t *F3T[MAXH][2];  // [240][256]
  const bf16_t *F3[MAXH][2];   // [240][256]
};

struct Workspace {
  int64_t cap = 0;            // atoms
  int cap_sys = 0;            // systems
  Grid *grids = nullptr;      // [cap_sys]  per-system cell grid (device)
  Grid *grids_host = nullptr; // [cap_sys]  pinned staging
  int *sys_off = nullptr;     // [cap_sys + 1]  first atom of each system (device); with one system
                              // and ghost atoms, [2..3] hold the centre range
  int *off_host = nullptr;    // pinned staging of sys_off
  int *sys_of = nullptr;      // [cap]  system of each atom
  int *slist = nullptr;       // [cap][SKIN_CAP]  skin list (within rc + skin)
  int *snnei = nullptr;       // [cap]
  double *xref = nullptr;     // [cap][3]  coordinates when the skin list was built
  int64_t skin_cap = 0;       // atoms the skin arrays hold
  int *cell_of = nullptr;     // [cap]
  int *cell_count = nullptr;  // [MAX_CELLS + 1]
  int *cell_start = nullptr;  // [MAX_CELLS + 1]
  int *cell_cursor = nullptr; // [MAX_CELLS]
  int *cell_atoms = nullptr;  // [cap]
  int *nlist = nullptr;       // [cap][SEL]
  int *nnei = nullptr;        // [cap]
  float *Gsave = nullptr;     // [cap][NATTN][GSAVE_LAYER]  inputs of each attention layer
  float *Tsave = nullptr;     // [cap][M][4]
  int *bidx = nullptr;        // [2][cap]  atoms of each backward kernel instance (bf16 path)
  int *bcnt = nullptr;        // [2]
  int *done = nullptr;        // [2 cap_sys + 1]  completion counters (the cell pass's workgroup counter
                              // at [2 cap_sys]); cleared at the start of each step
  float *D = nullptr;         // [cap][ND]  descriptor, then dE/dD
  double *Ei = nullptr;       // [cap] atomic energies (the weighted head combination)
  double *Eh = nullptr;       // [cap][MAXH]  atomic energy of each fitting head (models with several)
  double *Ehsys = nullptr;    // [cap_sys][MAXH]  each head's energy per system
  float4 *g = nullptr;        // [cap][SEL]  dE_i/dDelta_ij
  double *vpart = nullptr;    // [cap][9]   per-atom virial
  double *red = nullptr;      // scratch for the compensated reductions
  unsigned *flags = nullptr;  // [4] status words: flags, overflow count, rev misses, spare
  unsigned *flags_host = nullptr;  // pinned mirror
  double *gE = nullptr;       // [1] scale of the backward pass
  hipStream_t side = nullptr;  // second stream of the bf16 backward (its instances run side by side)
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  uint64_t gen = 0;           // bumped on every (re)allocation: graphs captured before it are stale
};

// How the neighbour lists of a step are made.
enum ListMode { LISTS_FRESH = 0, LISTS_SKIN_BUILD = 1, LISTS_SKIN_REUSE = 2 };
constexpr int DP_RETRY = 100;  // internal: redo the step with fresh lists

// One step: nsys systems, atoms concatenated (system s owns atoms off[s] .. off[s+1]-1).
struct StepArgs {
  int64_t n = 0;
  int nsys = 1;
  const double *X = nullptr;
  const int *types = nullptr;
  double *energy = nullptr;       // [nsys]
  double *forces = nullptr;       // [n][3] or NULL
  double *virial = nullptr;       // [nsys][9] or NULL
  double *atom_energy = nullptr;  // [n] or NULL
  bool open_single = false;       // one open-boundary system (grid made on the device)
  int ncells = 0;                 // cells over all systems
  int lists = LISTS_FRESH;
  int64_t n_centres = -1;         // one system: only atoms 0 .. n_centres-1 are centres (E_i, g_ij);
                                  // the rest are neighbours only (ghosts).  -1: every atom
  // one system in chunks: this call evaluates the centres c0 .. c1-1 (c1 = -1: to the end);
  // the first chunk builds the cell list and clears the step's flags and counters, the last
  // gathers forces and reduces energy and virial.  Chunks of a system run in order on one
  // workspace; lists, E_i and g_ij of earlier chunks stay in it.
  int64_t c0 = 0, c1 = -1;
  bool first_chunk = true, last_chunk = true;
};

struct GraphKey {
  int lists;
  int open_single;
  int64_t n;
  const void *X, *types, *energy, *forces, *virial, *atom_energy, *stream;
  double box[3];
  uint64_t ws_gen;  // workspace generation the graph's buffers belong to
};
struct GraphEntry {
  GraphKey key;
  hipGraphExec_t exec = nullptr;
};

}  // namespace dp

struct dp_model {
  int device = 0;
  int prec = 0;
  double rc = 0, rcs = 0, ln_eps = 1e-5;
  int sel = 0, ntypes = 0;
  void *wbuf = nullptr;
  dp::Weights<float> wf{};   // float32 path (its Tables part is also what the bf16 kernels read)
  dp::WeightsB16 wp{};       // bfloat16 path only
  dp::Workspace ws;
  // state kept between dp_compute_device (energy only) and dp_backward_device
  int64_t fwd_natoms = 0;
  const double *fwd_coords = nullptr;
  const int32_t *fwd_types = nullptr;
  int fwd_lists = 0;
  bool fwd_valid = false;
  // neighbour-list reuse with a skin (dp_set_skin)
  double skin = 0.0;
  int rebuild_every = 10;
  bool skin_valid = false;
  int skin_age = 0;
  int64_t skin_n = 0;
  bool skin_open = false;
  double skin_box[9] = {};
  int64_t skin_builds = 0, skin_rebuilds_forced = 0;
  // centres evaluated in chunks of this many atoms (dp_set_chunk; 0 = all at once)
  int64_t chunk = 0;
  // step graphs (dp_set_graph)
  bool use_graph = false;
  dp::GraphEntry graphs[4];
  int graph_next = 0;
  hipStream_t own_stream = nullptr;
  hipEvent_t dep_ev = nullptr;
  // per-phase timing (dp_profile_enable)
  bool prof = false;
  hipEvent_t ev[8] = {};
  double prof_ms[8] = {};
  int64_t prof_calls[8] = {};
};

namespace dp {
void set_error(const std::string &s);

// Launchers (defined in the kernel translation units); all enqueue on `st` and read the
// per-system grids (ws.grids), atom ranges (ws.sys_off) and atom -> system map (ws.sys_of).
// Clears the step's counters and flags (and ncells_zero cell counts) and maps atoms to systems.
void launch_prologue(const Workspace &ws, int nsys, int n, int ncells_zero, bool clear_flags, hipStream_t st);
void launch_cells(const Workspace &ws, const double *coords, const int *types, int n, int ntypes, bool open_single,
                  int ncells_total, double cell_cutoff, hipStream_t st);
// Lists for the atoms i0 .. i1-1 with candidates among all n; those at or beyond ncen get
// empty lists (ghost atoms).
void launch_nlist(const Workspace &ws, const double *coords, int n, int i0, int i1, int ncen, double cutoff,
                  bool skin, hipStream_t st);
void launch_filter(const Workspace &ws, const double *coords, int n, double rc, hipStream_t st);
// For models that need complete lists: turns a truncation (overflow count > 0) into the
// FLAG_INCOMPLETE error, so that the step's later kernels write nothing.
void launch_require_complete(const Workspace &ws, hipStream_t st);
// slot[i][j] (n x SEL) = the position of i in the list of its j-th neighbour, or -1 (also
// for j past the end of i's list); the lists are sorted, so each is a binary search.
void launch_rev_slots(const Workspace &ws, int n, int *slot, hipStream_t st);
void launch_skin_check(const Workspace &ws, const double *coords, const int *types, int n, int ntypes, double lim2,
                       hipStream_t st);
void launch_skin_ref(const Workspace &ws, const double *coords, int n, hipStream_t st);
// The per-centre launchers run over the centre atoms c0 .. c1-1, reading the coordinates
// and types of all n atoms as neighbours.
template <typename T>
void launch_descriptor_fwd(const Weights<T> &w, const Workspace &ws, const double *coords, const int *types,
                           int n, int c0, int c1, float rc, float rcs, float ln_eps, hipStream_t st);
// The fitting net over the first n atoms (E_i, and dE/dD over D when backward).
template <typename T>
void launch_fitting(const Weights<T> &w, const Workspace &ws, const int *types, int c0, int c1, bool backward,
                    hipStream_t st);
void launch_descriptor_fwd_b16(const Tables &w, const WeightsB16 &wp, const Workspace &ws,
                               const double *coords, const int *types, int n, int c0, int c1, float rc,
                               float rcs, float ln_eps, hipStream_t st);
void launch_descriptor_bwd_b16(const Tables &w, const WeightsB16 &wp, const Workspace &ws,
                               const double *coords, const int *types, int n, int c0, int c1, float rc,
                               float rcs, float ln_eps, hipStream_t st);
void launch_fitting_b16(const Tables &w, const WeightsB16 &wp, const Workspace &ws, const int *types, int c0,
                        int c1, bool backward, hipStream_t st);
template <typename T>
void launch_descriptor_bwd(const Weights<T> &w, const Workspace &ws, const double *coords, const int *types,
                           int n, int c0, int c1, float rc, float rcs, float ln_eps, hipStream_t st);
// Forces of all n atoms and the per-atom virial partials.  skin_rows: the step reused skin
// lists (one-sided pairs are then found through the skin rows, else through the cell list
// of the step); ghosts: atoms without lists are present.
void launch_forces(const Workspace &ws, const double *coords, int n, const double *gE, double *forces,
                   bool skin_rows, bool ghosts, hipStream_t st);
// Per-system energies (E_i over the device ranges eoff) and, if virial, virials (vpart over
// ws.sys_off), float64 Neumaier in a fixed order; energy and atom_energy may be NULL.
void launch_reduce(const Workspace &ws, const int *eoff, int nsys, double *energy, double *atom_energy,
                   double *virial, int nheads, hipStream_t st);
// out[0] = Neumaier sum of src over the atoms of system 0 (fixed order).
void launch_sum(const Workspace &ws, const double *src, double *out, hipStream_t st);

// Step orchestration (api.hip), shared with the serving loop.
size_t ws_bytes_per_atom(int prec);
// lists_only: only what the neighbour search, force gather and reductions use (no
// attention-descriptor buffers).
int ensure_ws(Workspace &ws, int prec, int64_t n, int nsys, bool skin, bool lists_only = false);
void free_ws(Workspace &ws);
int enqueue_step(dp_model *m, Workspace &ws, const StepArgs &a, hipStream_t st, bool profile);
int step_status(const Workspace &ws);
int make_grid(double rc, double cutoff, const double *box, Grid &g);
}  // namespace dp
