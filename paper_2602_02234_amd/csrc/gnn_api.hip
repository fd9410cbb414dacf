// C ABI of the GNN-variant model (declared in include/dp.h): model file, device
// weights, per-step buffers and the launch order of one energy/force/virial step.
// The neighbour search, force gather and float64 reductions are the library's shared
// kernels; the message-passing layers are in gnn.hip.
#include <cmath>
#include <cstring>
#include <fstream>
#include <string>
#include <vector>

#include "../../include/dp.h"
#include "gnn.h"

using namespace dp;

struct dp_gnn {
  int device = 0;
  int prec = 0;
  double rc = 0, rcs = 0, rca = 0;
  int sel = 0, asel = 0, ntypes = 0;
  void *wbuf = nullptr;
  gnn::Weights w{};
  Workspace ws;
  gnn::Buffers b;
  double *fpark = nullptr;  // forces when only the virial is asked for
  int64_t fpark_cap = 0;
  int64_t *tot_host = nullptr;  // pinned: angles, edges, angle-list edges
  int64_t last_angles = 0, last_edges = 0, last_aedges = 0;
  // per-phase device time (dp_gnn_profile_enable): lists, forward layers, backward
  // layers, forces and reductions
  bool prof = false;
  hipEvent_t ev[5] = {};
  double prof_ms[4] = {};
  int64_t prof_calls[4] = {};
  double lists_ms = 0.0;
};

namespace {

#define G_TRY(expr)                                                                        \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) {                                                                \
      set_error(std::string(#expr) + ": " + hipGetErrorString(e_));                        \
      return e_ == hipErrorOutOfMemory ? DP_ERR_OOM : DP_ERR_HIP;                          \
    }                                                                                      \
  } while (0)

using gnn::ADIM;
using gnn::EDIM;
using gnn::FWID;
using gnn::NDIM;
using gnn::NLAYER;

// (name, element count) of every array of the file, in file order.
std::vector<std::pair<std::string, size_t>> gnn_arrays(int ntypes) {
  std::vector<std::pair<std::string, size_t>> v = {
      {"TN", (size_t)ntypes * NDIM}, {"We0", EDIM}, {"be0", EDIM}, {"Wa0", ADIM}, {"ba0", ADIM}};
  for (int l = 0; l < NLAYER; ++l) {
    const std::string s = std::to_string(l);
    v.push_back({"Waa" + s, (size_t)(ADIM + 64) * ADIM});
    v.push_back({"baa" + s, ADIM});
    v.push_back({"Wea" + s, (size_t)(ADIM + 32) * EDIM});
    v.push_back({"bea" + s, EDIM});
    v.push_back({"Wee" + s, (size_t)(2 * NDIM + EDIM) * EDIM});
    v.push_back({"bee" + s, EDIM});
    v.push_back({"Wnn" + s, (size_t)(NDIM + EDIM) * NDIM});
    v.push_back({"bnn" + s, NDIM});
  }
  v.push_back({"G1", (size_t)NDIM * FWID});
  v.push_back({"d1", FWID});
  v.push_back({"G2", (size_t)FWID * FWID});
  v.push_back({"d2", FWID});
  v.push_back({"G3", FWID});
  v.push_back({"d3", 1});
  return v;
}

int load_weights(dp_gnn *m, const char *path) {
  std::ifstream f(path, std::ios::binary);
  if (!f) {
    set_error(std::string("cannot open GNN model file ") + path);
    return DP_ERR_MODEL_FILE;
  }
  std::vector<char> raw((std::istreambuf_iterator<char>(f)), std::istreambuf_iterator<char>());
  if (raw.size() < 128 || std::memcmp(raw.data(), "DPGNNv01", 8) != 0) {
    set_error("GNN model file: bad magic or short header");
    return DP_ERR_MODEL_FILE;
  }
  int32_t iv[16];
  double dv[4];
  std::memcpy(iv, raw.data() + 8, 64);
  std::memcpy(dv, raw.data() + 72, 32);
  if (iv[0] != 1 || iv[1] != NTYPES || iv[2] != NDIM || iv[3] != EDIM || iv[4] != ADIM || iv[5] != NLAYER ||
      iv[6] != FWID || iv[7] != SEL || iv[8] < 2 || iv[8] > gnn::ASEL) {
    set_error("GNN model file: version or dimensions differ from the compiled kernels");
    return DP_ERR_MODEL_FILE;
  }
  m->ntypes = iv[1];
  m->sel = iv[7];
  m->asel = iv[8];
  m->rc = dv[0];
  m->rcs = dv[1];
  m->rca = dv[2];
  if (!(m->rc > m->rcs && m->rcs > 0 && m->rca > m->rcs && m->rca <= m->rc)) {
    set_error("GNN model file: need 0 < rcs < rca <= rc");
    return DP_ERR_MODEL_FILE;
  }
  // device image: every array as float32 (256-byte aligned), plus G3 in float64
  std::vector<unsigned char> img;
  std::vector<size_t> offs;
  size_t off = 128;
  double d3 = 0.0;
  std::vector<double> G3;
  for (auto &a : gnn_arrays(m->ntypes)) {
    if (off + 8 * a.second > raw.size()) {
      set_error("GNN model file: truncated at " + a.first);
      return DP_ERR_MODEL_FILE;
    }
    std::vector<double> v(a.second);
    std::memcpy(v.data(), raw.data() + off, 8 * a.second);
    off += 8 * a.second;
    for (double x : v)
      if (!std::isfinite(x)) {
        set_error("GNN model file: non-finite value in " + a.first);
        return DP_ERR_MODEL_FILE;
      }
    if (a.first == "d3") d3 = v[0];
    if (a.first == "G3") G3 = v;
    const size_t o = (img.size() + 255) & ~size_t(255);
    img.resize(o + 4 * v.size());
    for (size_t k = 0; k < v.size(); ++k) {
      const float x = (float)v[k];
      std::memcpy(img.data() + o + 4 * k, &x, 4);
    }
    offs.push_back(o);
  }
  if (off != raw.size()) {
    set_error("GNN model file: size does not match its header");
    return DP_ERR_MODEL_FILE;
  }
  const size_t og = (img.size() + 255) & ~size_t(255);
  img.resize(og + 8 * FWID);
  std::memcpy(img.data() + og, G3.data(), 8 * FWID);
  G_TRY(hipMalloc(&m->wbuf, img.size()));
  G_TRY(hipMemcpy(m->wbuf, img.data(), img.size(), hipMemcpyHostToDevice));
  const unsigned char *base = (const unsigned char *)m->wbuf;
  size_t k = 0;
  auto nxt = [&]() { return (const float *)(base + offs[k++]); };
  gnn::Weights &w = m->w;
  w.TN = nxt(); w.We0 = nxt(); w.be0 = nxt(); w.Wa0 = nxt(); w.ba0 = nxt();
  for (int l = 0; l < NLAYER; ++l) {
    w.Waa[l] = nxt(); w.baa[l] = nxt(); w.Wea[l] = nxt(); w.bea[l] = nxt();
    w.Wee[l] = nxt(); w.bee[l] = nxt(); w.Wnn[l] = nxt(); w.bnn[l] = nxt();
  }
  w.G1 = nxt(); w.d1 = nxt(); w.G2 = nxt(); w.d2 = nxt(); w.G3 = nxt();
  (void)nxt();  // d3 goes by value
  w.G3d = (const double *)(base + og);
  w.d3 = d3;
  return DP_OK;
}

void free_buffers(gnn::Buffers &b) {
  void *ps[] = {b.aoff, b.nf, b.ef, b.af, b.da, b.de, b.dnj, b.dnl, b.gs, b.slot};
  for (void *p : ps)
    if (p) (void)hipFree(p);
  b = gnn::Buffers{};
}

int ensure_atoms(gnn::Buffers &b, int64_t n) {
  if (n <= b.cap) return DP_OK;
  const int64_t cap = std::max<int64_t>(n, b.cap + b.cap / 4);
  void *ps[] = {b.aoff, b.nf, b.ef, b.de, b.dnj, b.dnl, b.gs, b.slot};
  for (void *p : ps)
    if (p) (void)hipFree(p);
  b.aoff = nullptr; b.nf = b.ef = b.de = b.dnj = b.dnl = b.gs = nullptr;
  b.slot = nullptr;
  b.cap = 0;
  const size_t c = (size_t)cap, e = c * SEL * EDIM;
  G_TRY(hipMalloc(&b.aoff, (c + 3) * sizeof(int64_t)));
  G_TRY(hipMalloc(&b.nf, 2 * c * NDIM * sizeof(float)));
  G_TRY(hipMalloc(&b.ef, 3 * e * sizeof(float)));
  G_TRY(hipMalloc(&b.de, e * sizeof(float)));
  G_TRY(hipMalloc(&b.dnj, 2 * e * sizeof(float)));
  G_TRY(hipMalloc(&b.dnl, c * NDIM * sizeof(float)));
  G_TRY(hipMalloc(&b.gs, c * SEL * 2 * sizeof(float)));
  G_TRY(hipMalloc(&b.slot, c * SEL * sizeof(int)));
  b.cap = cap;
  return DP_OK;
}

int ensure_angles(gnn::Buffers &b, int64_t na) {
  if (na <= b.acap) return DP_OK;
  const int64_t cap = std::max<int64_t>(na, b.acap + b.acap / 4);
  if (b.af) (void)hipFree(b.af);
  if (b.da) (void)hipFree(b.da);
  b.af = b.da = nullptr;
  b.acap = 0;
  G_TRY(hipMalloc(&b.af, 3 * (size_t)cap * ADIM * sizeof(float)));
  G_TRY(hipMalloc(&b.da, (size_t)cap * ADIM * sizeof(float)));
  b.acap = cap;
  return DP_OK;
}

int gnn_status(const Workspace &ws) {
  const int s = step_status(ws);
  if (s == DP_WARN_SEL_OVERFLOW) {
    set_error("an atom has more than sel neighbours within rc; the message-passing model needs complete lists");
    return DP_ERR_TOO_LARGE;
  }
  return s;
}

int gnn_step(dp_gnn *m, int64_t natoms, const double *X, const int32_t *types, const double *box, double *energy,
             double *forces, double *virial, double *atom_energy, hipStream_t st) {
  Workspace &ws = m->ws;
  const int n = (int)natoms;
  Grid g;
  int s = make_grid(m->rc, m->rc, box, g);
  if (s != DP_OK) return s;
  s = ensure_ws(ws, m->prec, n, 1, false, true);
  if (s != DP_OK) return s;
  s = ensure_atoms(m->b, n);
  if (s != DP_OK) return s;
  const bool open = box == nullptr;
  const int ncells = open ? MAX_CELLS : g.ncells;
  ws.grids_host[0] = g;
  ws.off_host[0] = 0;
  ws.off_host[1] = n;
  if (!open) G_TRY(hipMemcpyAsync(ws.grids, ws.grids_host, sizeof(Grid), hipMemcpyHostToDevice, st));
  G_TRY(hipMemcpyAsync(ws.sys_off, ws.off_host, 2 * sizeof(int), hipMemcpyHostToDevice, st));
  if (m->prof) G_TRY(hipEventRecord(m->ev[0], st));
  launch_prologue(ws, 1, n, ncells + 1, true, st);
  launch_cells(ws, X, types, n, m->ntypes, open, ncells, m->rc, st);
  launch_nlist(ws, X, n, 0, n, n, m->rc, false, st);
  launch_require_complete(ws, st);
  gnn::Geo geo{(float)m->rc, (float)m->rcs, (float)m->rca, 1.f / (float)m->sel, 1.f / (float)m->asel, m->asel};
  gnn::launch_angle_offsets(m->b, ws, X, n, geo, st);
  G_TRY(hipGetLastError());
  if (m->prof) G_TRY(hipEventRecord(m->ev[1], st));
  // the angle count sizes the angle buffers: one host round trip per step
  G_TRY(hipMemcpyAsync(m->tot_host, m->b.aoff + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  G_TRY(hipMemcpyAsync(m->tot_host + 1, m->b.aoff + m->b.cap + 1, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, st));
  G_TRY(hipMemcpyAsync(ws.flags_host, ws.flags, 4 * sizeof(unsigned), hipMemcpyDeviceToHost, st));
  G_TRY(hipStreamSynchronize(st));
  if (m->prof) {
    float ms = 0.f;
    m->lists_ms = hipEventElapsedTime(&ms, m->ev[0], m->ev[1]) == hipSuccess ? ms : 0.0;
  }
  s = gnn_status(ws);
  if (s != DP_OK) return s;
  const int64_t na = m->tot_host[0];
  m->last_angles = na;
  m->last_edges = m->tot_host[1];
  m->last_aedges = m->tot_host[2];
  s = ensure_angles(m->b, std::max<int64_t>(na, 1));
  if (s != DP_OK) return s;
  const bool bwd = forces || virial;
  if (m->prof) G_TRY(hipEventRecord(m->ev[2], st));
  for (int l = 0; l < NLAYER; ++l) {
    if (m->prec == DP_BF16)
      gnn::launch_layer_fwd<bf16_t>(m->w, m->b, ws, X, types, n, l, geo, ws.Ei, st);
    else
      gnn::launch_layer_fwd<float>(m->w, m->b, ws, X, types, n, l, geo, ws.Ei, st);
  }
  if (m->prof) G_TRY(hipEventRecord(m->ev[3], st));
  if (bwd) {
    launch_rev_slots(ws, n, m->b.slot, st);
    for (int l = NLAYER - 1; l >= 0; --l) {
      if (m->prec == DP_BF16)
        gnn::launch_layer_bwd<bf16_t>(m->w, m->b, ws, X, types, n, l, geo, st);
      else
        gnn::launch_layer_bwd<float>(m->w, m->b, ws, X, types, n, l, geo, st);
    }
  }
  if (m->prof) G_TRY(hipEventRecord(m->ev[4], st));
  if (bwd) {
    double *F = forces;
    if (!F) {
      if (m->fpark_cap < n) {
        if (m->fpark) (void)hipFree(m->fpark);
        m->fpark = nullptr;
        m->fpark_cap = 0;
        G_TRY(hipMalloc(&m->fpark, (size_t)n * 3 * sizeof(double)));
        m->fpark_cap = n;
      }
      F = m->fpark;
    }
    launch_forces(ws, X, n, nullptr, F, false, false, st);
  }
  launch_reduce(ws, ws.sys_off, 1, energy, atom_energy, virial, 1, st);
  G_TRY(hipGetLastError());
  if (m->prof) G_TRY(hipEventRecord(m->ev[0], st));  // end of the last phase (ev[0] is free again)
  G_TRY(hipMemcpyAsync(ws.flags_host, ws.flags, 4 * sizeof(unsigned), hipMemcpyDeviceToHost, st));
  G_TRY(hipStreamSynchronize(st));
  s = gnn_status(ws);
  if (s >= 0 && m->prof) {
    // phases: lists ev1 - (start), fwd ev3 - ev2, bwd ev4 - ev3, forces/reductions end - ev4
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, m->ev[2], m->ev[3]) == hipSuccess) { m->prof_ms[1] += ms; m->prof_calls[1] += 1; }
    if (bwd && hipEventElapsedTime(&ms, m->ev[3], m->ev[4]) == hipSuccess) {
      m->prof_ms[2] += ms;
      m->prof_calls[2] += 1;
    }
    if (hipEventElapsedTime(&ms, m->ev[4], m->ev[0]) == hipSuccess) { m->prof_ms[3] += ms; m->prof_calls[3] += 1; }
    m->prof_ms[0] += m->lists_ms;
    m->prof_calls[0] += 1;
  }
  return s;
}

}  // namespace

extern "C" {

int dp_gnn_load(const char *path, int precision, int device, dp_gnn **out) {
  set_error("");
  if (!path || !out || (precision != DP_FP32 && precision != DP_BF16)) {
    set_error("dp_gnn_load: bad argument");
    return DP_ERR_ARG;
  }
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    set_error("dp_gnn_load: no such device");
    return DP_ERR_ARG;
  }
  G_TRY(hipSetDevice(device));
  dp_gnn *m = new dp_gnn();
  m->device = device;
  m->prec = precision;
  int s = load_weights(m, path);
  if (s == DP_OK && hipHostMalloc(&m->tot_host, 3 * sizeof(int64_t), hipHostMallocDefault) != hipSuccess) {
    set_error("dp_gnn_load: pinned allocation failed");
    s = DP_ERR_OOM;
  }
  if (s != DP_OK) {
    dp_gnn_free(m);
    return s;
  }
  *out = m;
  return DP_OK;
}

void dp_gnn_free(dp_gnn *m) {
  if (!m) return;
  (void)hipSetDevice(m->device);
  (void)hipDeviceSynchronize();
  free_buffers(m->b);
  free_ws(m->ws);
  if (m->fpark) (void)hipFree(m->fpark);
  if (m->wbuf) (void)hipFree(m->wbuf);
  if (m->tot_host) (void)hipHostFree(m->tot_host);
  for (auto &e : m->ev)
    if (e) (void)hipEventDestroy(e);
  delete m;
}

int dp_gnn_info(const dp_gnn *m, double *rc, double *rca, int *sel, int *asel) {
  if (!m) {
    set_error("dp_gnn_info: bad argument");
    return DP_ERR_ARG;
  }
  if (rc) *rc = m->rc;
  if (rca) *rca = m->rca;
  if (sel) *sel = m->sel;
  if (asel) *asel = m->asel;
  return DP_OK;
}

int dp_gnn_compute_device(dp_gnn *m, int64_t natoms, const double *d_coords, const int32_t *d_types,
                          const double *box_host, double *d_energy, double *d_forces, double *d_virial,
                          double *d_atom_energy, void *hip_stream) {
  set_error("");
  if (!m || natoms < 1 || !d_coords || !d_types || !d_energy) {
    set_error("dp_gnn_compute_device: bad argument");
    return DP_ERR_ARG;
  }
  if (natoms > (1 << 24)) {
    set_error("natoms above the library limit");
    return DP_ERR_TOO_LARGE;
  }
  G_TRY(hipSetDevice(m->device));
  return gnn_step(m, natoms, d_coords, d_types, box_host, d_energy, d_forces, d_virial, d_atom_energy,
                  (hipStream_t)hip_stream);
}

int dp_gnn_graph_size(const dp_gnn *m, int64_t *edges, int64_t *angle_edges, int64_t *angles) {
  if (!m) {
    set_error("dp_gnn_graph_size: bad argument");
    return DP_ERR_ARG;
  }
  if (edges) *edges = m->last_edges;
  if (angle_edges) *angle_edges = m->last_aedges;
  if (angles) *angles = m->last_angles;
  return DP_OK;
}

int dp_gnn_profile_enable(dp_gnn *m, int enable) {
  if (!m) {
    set_error("dp_gnn_profile_enable: bad argument");
    return DP_ERR_ARG;
  }
  G_TRY(hipSetDevice(m->device));
  if (enable && !m->ev[0])
    for (auto &e : m->ev) G_TRY(hipEventCreate(&e));
  m->prof = enable != 0;
  for (int k = 0; k < 4; ++k) {
    m->prof_ms[k] = 0.0;
    m->prof_calls[k] = 0;
  }
  return DP_OK;
}

int dp_gnn_profile_read(const dp_gnn *m, double *ms, int64_t *calls, int max) {
  if (!m || !ms || !calls || max < 0) {
    set_error("dp_gnn_profile_read: bad argument");
    return DP_ERR_ARG;
  }
  const int k = max < 4 ? max : 4;
  for (int q = 0; q < k; ++q) {
    ms[q] = m->prof_ms[q];
    calls[q] = m->prof_calls[q];
  }
  return k;
}

}  // extern "C"
