// C ABI of the repformer-style model (declared in include/dp.h): model file, device
// weights, per-step buffers and the launch order of one energy/force/virial step.  The
// neighbour search, force gather and float64 reductions are the library's shared kernels;
// the layers are in repformer.hip.
#include <cmath>
#include <cstring>
#include <fstream>
#include <string>
#include <vector>

#include "../../include/dp.h"
#include "repformer.h"

using namespace dp;

struct dp_rep {
  int device = 0;
  double rc = 0, rcs = 0;
  int sel = 0, ntypes = 0;
  void *wbuf = nullptr;
  rep::Weights w{};
  Workspace ws;
  rep::Buffers b;
  double *fpark = nullptr;
  int64_t fpark_cap = 0;
  int64_t *etot_host = nullptr;
  int64_t last_edges = 0;
  // per-phase device time (dp_rep_profile_enable): lists, forward layers, backward layers,
  // forces and reductions
  bool prof = false;
  hipEvent_t ev[5] = {};
  double prof_ms[4] = {};
  int64_t prof_calls[4] = {};
};

namespace {

#define R_TRY(expr)                                                                        \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) {                                                                \
      set_error(std::string(#expr) + ": " + hipGetErrorString(e_));                        \
      return e_ == hipErrorOutOfMemory ? DP_ERR_OOM : DP_ERR_HIP;                          \
    }                                                                                      \
  } while (0)

using rep::FWID;
using rep::G1D;
using rep::G2D;
using rep::NLAYER;
using rep::XD;

std::vector<std::pair<std::string, size_t>> rep_arrays(int ntypes) {
  std::vector<std::pair<std::string, size_t>> v = {{"TN", (size_t)ntypes * G1D}, {"Wp0", G2D}, {"bp0", G2D}};
  for (int l = 0; l < NLAYER; ++l) {
    const std::string s = std::to_string(l);
    v.push_back({"Wa" + s, (size_t)(G2D + G1D) * G2D});
    v.push_back({"ba" + s, G2D});
    v.push_back({"Wq" + s, (size_t)G2D * G2D});
    v.push_back({"Wk" + s, (size_t)G2D * G2D});
    v.push_back({"Wv" + s, (size_t)G2D * G2D});
    v.push_back({"W1" + s, (size_t)XD * G1D});
    v.push_back({"b1" + s, G1D});
  }
  v.push_back({"G1", (size_t)G1D * FWID});
  v.push_back({"d1", FWID});
  v.push_back({"G2", (size_t)FWID * FWID});
  v.push_back({"d2", FWID});
  v.push_back({"G3", FWID});
  v.push_back({"d3", 1});
  return v;
}

int load_weights(dp_rep *m, const char *path) {
  std::ifstream f(path, std::ios::binary);
  if (!f) {
    set_error(std::string("cannot open repformer model file ") + path);
    return DP_ERR_MODEL_FILE;
  }
  std::vector<char> raw((std::istreambuf_iterator<char>(f)), std::istreambuf_iterator<char>());
  if (raw.size() < 128 || std::memcmp(raw.data(), "DPREPv01", 8) != 0) {
    set_error("repformer model file: bad magic or short header");
    return DP_ERR_MODEL_FILE;
  }
  int32_t iv[16];
  double dv[3];
  std::memcpy(iv, raw.data() + 8, 64);
  std::memcpy(dv, raw.data() + 72, 24);
  if (iv[0] != 1 || iv[1] != NTYPES || iv[2] != G1D || iv[3] != G2D || iv[4] != rep::NAX || iv[5] != NLAYER ||
      iv[6] != FWID || iv[7] != SEL) {
    set_error("repformer model file: version or dimensions differ from the compiled kernels");
    return DP_ERR_MODEL_FILE;
  }
  m->ntypes = iv[1];
  m->sel = iv[7];
  m->rc = dv[0];
  m->rcs = dv[1];
  if (!(m->rc > m->rcs && m->rcs > 0)) {
    set_error("repformer model file: need 0 < rcs < rc");
    return DP_ERR_MODEL_FILE;
  }
  std::vector<unsigned char> img;
  std::vector<size_t> offs;
  size_t off = 128;
  double d3 = 0.0;
  std::vector<double> G3;
  for (auto &a : rep_arrays(m->ntypes)) {
    if (off + 8 * a.second > raw.size()) {
      set_error("repformer model file: truncated at " + a.first);
      return DP_ERR_MODEL_FILE;
    }
    std::vector<double> v(a.second);
    std::memcpy(v.data(), raw.data() + off, 8 * a.second);
    off += 8 * a.second;
    for (double x : v)
      if (!std::isfinite(x)) {
        set_error("repformer model file: non-finite value in " + a.first);
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
    set_error("repformer model file: size does not match its header");
    return DP_ERR_MODEL_FILE;
  }
  const size_t og = (img.size() + 255) & ~size_t(255);
  img.resize(og + 8 * FWID);
  std::memcpy(img.data() + og, G3.data(), 8 * FWID);
  R_TRY(hipMalloc(&m->wbuf, img.size()));
  R_TRY(hipMemcpy(m->wbuf, img.data(), img.size(), hipMemcpyHostToDevice));
  const unsigned char *base = (const unsigned char *)m->wbuf;
  size_t k = 0;
  auto nxt = [&]() { return (const float *)(base + offs[k++]); };
  rep::Weights &w = m->w;
  w.TN = nxt(); w.Wp0 = nxt(); w.bp0 = nxt();
  for (int l = 0; l < NLAYER; ++l) {
    w.Wa[l] = nxt(); w.ba[l] = nxt(); w.Wq[l] = nxt(); w.Wk[l] = nxt(); w.Wv[l] = nxt();
    w.W1[l] = nxt(); w.b1[l] = nxt();
  }
  w.G1 = nxt(); w.d1 = nxt(); w.G2 = nxt(); w.d2 = nxt(); w.G3 = nxt();
  (void)nxt();  // d3 goes by value
  w.G3d = (const double *)(base + og);
  w.d3 = d3;
  return DP_OK;
}

void free_buffers(rep::Buffers &b) {
  void *ps[] = {b.g1f, b.g2f, b.dg2, b.dnj, b.dnl, b.gs, b.slot, b.etot};
  for (void *p : ps)
    if (p) (void)hipFree(p);
  b = rep::Buffers{};
}

int ensure_buffers(rep::Buffers &b, int64_t n) {
  if (!b.etot) R_TRY(hipMalloc(&b.etot, sizeof(int64_t)));
  if (n <= b.cap) return DP_OK;
  const int64_t cap = std::max<int64_t>(n, b.cap + b.cap / 4);
  void *ps[] = {b.g1f, b.g2f, b.dg2, b.dnj, b.dnl, b.gs, b.slot};
  for (void *p : ps)
    if (p) (void)hipFree(p);
  b.g1f = b.g2f = b.dg2 = b.dnj = b.dnl = b.gs = nullptr;
  b.slot = nullptr;
  b.cap = 0;
  const size_t c = (size_t)cap, e = c * SEL;
  R_TRY(hipMalloc(&b.g1f, 2 * c * G1D * sizeof(float)));
  R_TRY(hipMalloc(&b.g2f, 3 * e * G2D * sizeof(float)));
  R_TRY(hipMalloc(&b.dg2, e * G2D * sizeof(float)));
  R_TRY(hipMalloc(&b.dnj, 2 * e * G1D * sizeof(float)));
  R_TRY(hipMalloc(&b.dnl, c * G1D * sizeof(float)));
  R_TRY(hipMalloc(&b.gs, e * rep::GSN * sizeof(float)));
  R_TRY(hipMalloc(&b.slot, e * sizeof(int)));
  b.cap = cap;
  return DP_OK;
}

int rep_status(const Workspace &ws) {
  const int s = step_status(ws);
  if (s == DP_WARN_SEL_OVERFLOW) {
    set_error("an atom has more than sel neighbours within rc; the message-passing model needs complete lists");
    return DP_ERR_TOO_LARGE;
  }
  return s;
}

void record(dp_rep *m, int k, hipStream_t st) {
  if (m->prof) (void)hipEventRecord(m->ev[k], st);
}

int rep_step(dp_rep *m, int64_t natoms, const double *X, const int32_t *types, const double *box, double *energy,
             double *forces, double *virial, double *atom_energy, hipStream_t st) {
  Workspace &ws = m->ws;
  const int n = (int)natoms;
  Grid g;
  int s = make_grid(m->rc, m->rc, box, g);
  if (s != DP_OK) return s;
  s = ensure_ws(ws, DP_FP32, n, 1, false, true);
  if (s != DP_OK) return s;
  s = ensure_buffers(m->b, n);
  if (s != DP_OK) return s;
  const bool open = box == nullptr;
  const int ncells = open ? MAX_CELLS : g.ncells;
  ws.grids_host[0] = g;
  ws.off_host[0] = 0;
  ws.off_host[1] = n;
  if (!open) R_TRY(hipMemcpyAsync(ws.grids, ws.grids_host, sizeof(Grid), hipMemcpyHostToDevice, st));
  R_TRY(hipMemcpyAsync(ws.sys_off, ws.off_host, 2 * sizeof(int), hipMemcpyHostToDevice, st));
  record(m, 0, st);
  launch_prologue(ws, 1, n, ncells + 1, true, st);
  launch_cells(ws, X, types, n, m->ntypes, open, ncells, m->rc, st);
  launch_nlist(ws, X, n, 0, n, n, m->rc, false, st);
  launch_require_complete(ws, st);
  rep::launch_edge_count(m->b, ws, n, st);
  record(m, 1, st);
  rep::Geo geo{(float)m->rc, (float)m->rcs, 1.f / (float)m->sel};
  for (int l = 0; l < NLAYER; ++l) rep::launch_layer_fwd(m->w, m->b, ws, X, types, n, l, geo, ws.Ei, st);
  record(m, 2, st);
  const bool bwd = forces || virial;
  if (bwd) {
    launch_rev_slots(ws, n, m->b.slot, st);
    for (int l = NLAYER - 1; l >= 0; --l) rep::launch_layer_bwd(m->w, m->b, ws, X, types, n, l, geo, st);
  }
  record(m, 3, st);
  if (bwd) {
    double *F = forces;
    if (!F) {
      if (m->fpark_cap < n) {
        if (m->fpark) (void)hipFree(m->fpark);
        m->fpark = nullptr;
        m->fpark_cap = 0;
        R_TRY(hipMalloc(&m->fpark, (size_t)n * 3 * sizeof(double)));
        m->fpark_cap = n;
      }
      F = m->fpark;
    }
    launch_forces(ws, X, n, nullptr, F, false, false, st);
  }
  launch_reduce(ws, ws.sys_off, 1, energy, atom_energy, virial, 1, st);
  record(m, 4, st);
  R_TRY(hipGetLastError());
  R_TRY(hipMemcpyAsync(m->etot_host, m->b.etot, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  R_TRY(hipMemcpyAsync(ws.flags_host, ws.flags, 4 * sizeof(unsigned), hipMemcpyDeviceToHost, st));
  R_TRY(hipStreamSynchronize(st));
  s = rep_status(ws);
  if (s < 0) return s;
  m->last_edges = *m->etot_host;
  if (m->prof)
    for (int k = 0; k < 4; ++k) {
      float ms = 0.f;
      if (k == 2 && !bwd) continue;
      if (hipEventElapsedTime(&ms, m->ev[k], m->ev[k + 1]) == hipSuccess) {
        m->prof_ms[k] += ms;
        m->prof_calls[k] += 1;
      }
    }
  return s;
}

}  // namespace

extern "C" {

int dp_rep_load(const char *path, int device, dp_rep **out) {
  set_error("");
  if (!path || !out) {
    set_error("dp_rep_load: bad argument");
    return DP_ERR_ARG;
  }
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    set_error("dp_rep_load: no such device");
    return DP_ERR_ARG;
  }
  R_TRY(hipSetDevice(device));
  dp_rep *m = new dp_rep();
  m->device = device;
  int s = load_weights(m, path);
  if (s == DP_OK && hipHostMalloc(&m->etot_host, sizeof(int64_t), hipHostMallocDefault) != hipSuccess) {
    set_error("dp_rep_load: pinned allocation failed");
    s = DP_ERR_OOM;
  }
  if (s != DP_OK) {
    dp_rep_free(m);
    return s;
  }
  *out = m;
  return DP_OK;
}

void dp_rep_free(dp_rep *m) {
  if (!m) return;
  (void)hipSetDevice(m->device);
  (void)hipDeviceSynchronize();
  free_buffers(m->b);
  free_ws(m->ws);
  if (m->fpark) (void)hipFree(m->fpark);
  if (m->wbuf) (void)hipFree(m->wbuf);
  if (m->etot_host) (void)hipHostFree(m->etot_host);
  for (auto &e : m->ev)
    if (e) (void)hipEventDestroy(e);
  delete m;
}

int dp_rep_compute_device(dp_rep *m, int64_t natoms, const double *d_coords, const int32_t *d_types,
                          const double *box_host, double *d_energy, double *d_forces, double *d_virial,
                          double *d_atom_energy, void *hip_stream) {
  set_error("");
  if (!m || natoms < 1 || !d_coords || !d_types || !d_energy) {
    set_error("dp_rep_compute_device: bad argument");
    return DP_ERR_ARG;
  }
  if (natoms > (1 << 24)) {
    set_error("natoms above the library limit");
    return DP_ERR_TOO_LARGE;
  }
  R_TRY(hipSetDevice(m->device));
  return rep_step(m, natoms, d_coords, d_types, box_host, d_energy, d_forces, d_virial, d_atom_energy,
                  (hipStream_t)hip_stream);
}

int dp_rep_edges(const dp_rep *m, int64_t *edges) {
  if (!m || !edges) {
    set_error("dp_rep_edges: bad argument");
    return DP_ERR_ARG;
  }
  *edges = m->last_edges;
  return DP_OK;
}

int dp_rep_profile_enable(dp_rep *m, int enable) {
  if (!m) {
    set_error("dp_rep_profile_enable: bad argument");
    return DP_ERR_ARG;
  }
  R_TRY(hipSetDevice(m->device));
  if (enable && !m->ev[0])
    for (auto &e : m->ev) R_TRY(hipEventCreate(&e));
  m->prof = enable != 0;
  for (int k = 0; k < 4; ++k) {
    m->prof_ms[k] = 0.0;
    m->prof_calls[k] = 0;
  }
  return DP_OK;
}

int dp_rep_profile_read(const dp_rep *m, double *ms, int64_t *calls, int max) {
  if (!m || !ms || !calls || max < 0) {
    set_error("dp_rep_profile_read: bad argument");
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
