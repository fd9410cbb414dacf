// C ABI of the library (declared in include/dp.h): model loading, argument
// validation, the device workspace and the order of the kernels of one step.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <mutex>
#include <type_traits>
#include <string>
#include <vector>

#include "../../include/dp.h"
#include "dp_internal.h"

namespace dp {

static thread_local std::string g_last_error;
void set_error(const std::string &s) { g_last_error = s; }

namespace {

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) {                                                                \
      set_error(std::string(#expr) + ": " + hipGetErrorString(e_));                        \
      return e_ == hipErrorOutOfMemory ? DP_ERR_OOM : DP_ERR_HIP;                          \
    }                                                                                      \
  } while (0)

uint16_t to_bf16(float f) {  // round to nearest even
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

struct HostModel {
  int ntypes, tebd, e1, e2, M_, natt, d, m2, fh, nfh, sel, nheads;
  double rc, rcs, eps, fscale;
  std::vector<double> TE, W1, b1, W2, b2, W3, b3;
  std::vector<double> WQ[NATTN], WK[NATTN], WV[NATTN], WO[NATTN], gam[NATTN], bet[NATTN];
  // per fitting head
  std::vector<double> F1[MAXH], c1[MAXH], F2[MAXH], c2[MAXH], F3[MAXH], c3[MAXH], F4[MAXH], c4[MAXH], ebias[MAXH];
};

int read_model(const char *path, HostModel &h) {
  std::ifstream f(path, std::ios::binary);
  if (!f) {
    set_error(std::string("cannot open model file ") + path);
    return DP_ERR_MODEL_FILE;
  }
  std::vector<char> raw((std::istreambuf_iterator<char>(f)), std::istreambuf_iterator<char>());
  if (raw.size() < 128 || std::memcmp(raw.data(), "DPAMDv01", 8) != 0) {
    set_error("model file: bad magic or short header");
    return DP_ERR_MODEL_FILE;
  }
  int32_t iv[16];
  std::memcpy(iv, raw.data() + 8, 64);
  double dv[4];
  std::memcpy(dv, raw.data() + 72, 32);
  if (iv[0] != 1) {
    set_error("model file: unsupported version");
    return DP_ERR_MODEL_FILE;
  }
  h.ntypes = iv[1]; h.tebd = iv[2]; h.e1 = iv[3]; h.e2 = iv[4]; h.M_ = iv[5]; h.natt = iv[6]; h.d = iv[7];
  h.m2 = iv[8]; h.fh = iv[9]; h.nfh = iv[10]; h.sel = iv[11];
  h.nheads = iv[12] > 1 ? iv[12] : 1;  // the first reserved int: number of fitting heads
  if (iv[12] < 0 || h.nheads > MAXH) {
    set_error("model file: more fitting heads than the library supports (" + std::to_string(MAXH) + ")");
    return DP_ERR_MODEL_FILE;
  }
  h.rc = dv[0]; h.rcs = dv[1]; h.eps = dv[2]; h.fscale = dv[3];
  if (h.ntypes != NTYPES || h.tebd != TEBD || h.e1 != E1 || h.e2 != E2 || h.M_ != M || h.natt != NATTN ||
      h.d != DATTN || h.m2 != M2 || h.fh != FH || h.nfh != 3 || h.sel != SEL) {
    set_error("model file: dimensions differ from the compiled kernels");
    return DP_ERR_MODEL_FILE;
  }
  if (!(h.rc > h.rcs && h.rcs > 0 && h.eps > 0)) {
    set_error("model file: bad rc/rcs/eps");
    return DP_ERR_MODEL_FILE;
  }
  size_t off = 128;
  bool bad = false;
  auto take = [&](std::vector<double> &v, size_t cnt) {
    if (off + 8 * cnt > raw.size()) { bad = true; return; }
    v.resize(cnt);
    std::memcpy(v.data(), raw.data() + off, 8 * cnt);
    off += 8 * cnt;
  };
  take(h.TE, NTYPES * TEBD);
  take(h.W1, (1 + 2 * TEBD) * E1); take(h.b1, E1);
  take(h.W2, E1 * E2); take(h.b2, E2);
  take(h.W3, E2 * M); take(h.b3, M);
  for (int a = 0; a < NATTN; ++a) {
    take(h.WQ[a], M * DATTN); take(h.WK[a], M * DATTN); take(h.WV[a], M * DATTN); take(h.WO[a], DATTN * M);
    take(h.gam[a], M); take(h.bet[a], M);
  }
  for (int k = 0; k < h.nheads; ++k) {
    take(h.F1[k], ND * FH); take(h.c1[k], FH);
    take(h.F2[k], FH * FH); take(h.c2[k], FH);
    take(h.F3[k], FH * FH); take(h.c3[k], FH);
    take(h.F4[k], FH); take(h.c4[k], 1);
    take(h.ebias[k], NTYPES);
  }
  if (bad || off != raw.size()) {
    set_error("model file: size does not match its header");
    return DP_ERR_MODEL_FILE;
  }
  return DP_OK;
}

// Device image of the weights: float tables + GEMM operands in T, 256-byte aligned pieces.
struct Packer {
  std::vector<unsigned char> bytes;
  size_t add(const void *p, size_t n) {
    size_t o = (bytes.size() + 255) & ~size_t(255);
    bytes.resize(o + n);
    std::memcpy(bytes.data() + o, p, n);
    return o;
  }
  size_t addf(const std::vector<float> &v) { return add(v.data(), v.size() * 4); }
  size_t addd(const std::vector<double> &v) { return add(v.data(), v.size() * 8); }
};

std::vector<float> tof(const std::vector<double> &v) { return std::vector<float>(v.begin(), v.end()); }
// [rows][cols] -> [cols][rows]
std::vector<float> transpose(const std::vector<double> &v, int rows, int cols) {
  std::vector<float> o((size_t)rows * cols);
  for (int r = 0; r < rows; ++r)
    for (int c = 0; c < cols; ++c) o[(size_t)c * rows + r] = (float)v[(size_t)r * cols + c];
  return o;
}

// Offsets of the pieces of the weight image, in the order the binders take them.
struct Image {
  Packer pk;
  std::vector<size_t> tab, f32, b16;
  int nheads = 1;
  double c4[MAXH] = {};
};

// The whole device weight image on the host (no HIP call): the tables both paths read,
// then the GEMM operands of the model's precision only.
void pack_weights(const HostModel &h, int pr, Image &im) {
  Packer &pk = im.pk;
  std::vector<size_t> &o = im.tab;
  // first embedding layer: s column, and the type part folded with the bias
  std::vector<float> w1s(E1), Bt(NTYPES * NTYPES * E1);
  for (int e = 0; e < E1; ++e) w1s[e] = (float)h.W1[e];
  for (int ti = 0; ti < NTYPES; ++ti)
    for (int tj = 0; tj < NTYPES; ++tj)
      for (int e = 0; e < E1; ++e) {
        double acc = h.b1[e];
        for (int q = 0; q < TEBD; ++q) {
          acc += h.TE[tj * TEBD + q] * h.W1[(1 + q) * E1 + e];
          acc += h.TE[ti * TEBD + q] * h.W1[(1 + TEBD + q) * E1 + e];
        }
        Bt[(ti * NTYPES + tj) * E1 + e] = (float)acc;
      }
  o.push_back(pk.addf(w1s));
  o.push_back(pk.addf(Bt));
  o.push_back(pk.addf(tof(h.b2)));
  o.push_back(pk.addf(tof(h.b3)));
  for (int a = 0; a < NATTN; ++a) {
    o.push_back(pk.addf(tof(h.gam[a])));
    o.push_back(pk.addf(tof(h.bet[a])));
  }
  im.nheads = h.nheads;
  for (int k = 0; k < h.nheads; ++k) {
    o.push_back(pk.addf(tof(h.c1[k])));
    o.push_back(pk.addf(tof(h.c2[k])));
    o.push_back(pk.addf(tof(h.c3[k])));
    o.push_back(pk.addf(tof(h.F4[k])));
    o.push_back(pk.addd(h.F4[k]));
    o.push_back(pk.addd(h.ebias[k]));
    im.c4[k] = h.c4[k][0];
  }
  // the fused single-head attention operands, formed in float64
  const double isd = 1.0 / std::sqrt((double)DATTN);
  std::vector<double> QK[NATTN], VO[NATTN];
  for (int a = 0; a < NATTN; ++a) {
    QK[a].assign((size_t)M * M, 0.0);
    VO[a].assign((size_t)M * M, 0.0);
    for (int r = 0; r < M; ++r)
      for (int c = 0; c < M; ++c) {
        double s1 = 0, s2 = 0;
        for (int q = 0; q < DATTN; ++q) {
          s1 += h.WQ[a][(size_t)r * DATTN + q] * h.WK[a][(size_t)c * DATTN + q];
          s2 += h.WV[a][(size_t)r * DATTN + q] * h.WO[a][(size_t)q * M + c];
        }
        QK[a][(size_t)r * M + c] = s1 * isd;
        VO[a][(size_t)r * M + c] = s2;
      }
  }
  if (pr == DP_FP32) {
    std::vector<size_t> &f = im.f32;
    f.push_back(pk.addf(transpose(h.W2, E1, E2)));
    f.push_back(pk.addf(tof(h.W2)));
    f.push_back(pk.addf(transpose(h.W3, E2, M)));
    f.push_back(pk.addf(tof(h.W3)));
    for (int a = 0; a < NATTN; ++a) {
      f.push_back(pk.addf(transpose(QK[a], M, M)));
      f.push_back(pk.addf(tof(QK[a])));
      f.push_back(pk.addf(transpose(VO[a], M, M)));
      f.push_back(pk.addf(tof(VO[a])));
    }
    for (int k = 0; k < h.nheads; ++k) {
      f.push_back(pk.addf(transpose(h.F1[k], ND, FH)));
      f.push_back(pk.addf(tof(h.F1[k])));
      f.push_back(pk.addf(transpose(h.F2[k], FH, FH)));
      f.push_back(pk.addf(tof(h.F2[k])));
      f.push_back(pk.addf(transpose(h.F3[k], FH, FH)));
      f.push_back(pk.addf(tof(h.F3[k])));
    }
    return;
  }
  // padded [rows][k] bf16 operands of the bfloat16 kernels (zero outside the real extent)
  std::vector<size_t> &op = im.b16;
  auto mat = [](int R, int K, auto f) {
    std::vector<float> v((size_t)R * K, 0.f);
    for (int r = 0; r < R; ++r)
      for (int k = 0; k < K; ++k) v[(size_t)r * K + k] = (float)f(r, k);
    return v;
  };
  auto hi_lo = [&](const std::vector<float> &v, int part) {
    std::vector<uint16_t> b(v.size());
    for (size_t i = 0; i < v.size(); ++i) {
      const uint16_t hb = to_bf16(v[i]);
      uint32_t hu = (uint32_t)hb << 16;
      float hf;
      std::memcpy(&hf, &hu, 4);
      b[i] = part == 0 ? hb : to_bf16(v[i] - hf);
    }
    return pk.add(b.data(), b.size() * 2);
  };
  auto W2 = [&](int a, int b) { return h.W2[(size_t)a * E2 + b]; };
  auto W3 = [&](int a, int b) { return h.W3[(size_t)a * M + b]; };
  op.push_back(hi_lo(mat(64, 32, [&](int c, int k) { return (c < E2 && k < E1) ? W2(k, c) : 0.0; }), 0));
  op.push_back(hi_lo(mat(112, 64, [&](int c, int k) { return (c < M && k < E2) ? W3(k, c) : 0.0; }), 0));
  op.push_back(hi_lo(mat(64, 112, [&](int c, int k) { return (c < E2 && k < M) ? W3(c, k) : 0.0; }), 0));
  op.push_back(hi_lo(mat(32, 64, [&](int c, int k) { return (c < E1 && k < E2) ? W2(c, k) : 0.0; }), 0));
  for (int a = 0; a < NATTN; ++a) {
    const std::vector<double> &qk = QK[a], &vo = VO[a];
    auto at = [](const std::vector<double> &v, int r, int c) { return (r < M && c < M) ? v[(size_t)r * M + c] : 0.0; };
    // the attention products read these from global memory, in MFMA fragment order: per 16-column tile, three 32-k fragments of 64 lanes x 8 values (lane l:
    // row l % 16, k = 32 s + 8 (l / 16) ..), then the k = 96..111 tail as 64 lanes x 4
    auto frag112 = [](const std::vector<float> &v) {
      std::vector<float> o(v.size());
      for (int t = 0; t < 7; ++t)
        for (int l = 0; l < 64; ++l) {
          const size_t row = (size_t)(16 * t + l % 16) * 112;
          for (int st = 0; st < 3; ++st)
            for (int e = 0; e < 8; ++e) o[t * 1792 + st * 512 + l * 8 + e] = v[row + 32 * st + 8 * (l / 16) + e];
          for (int e = 0; e < 4; ++e) o[t * 1792 + 1536 + l * 4 + e] = v[row + 96 + 4 * (l / 16) + e];
        }
      return o;
    };
    op.push_back(hi_lo(frag112(mat(112, 112, [&](int c, int k) { return at(qk, k, c); })), 0));
    op.push_back(hi_lo(frag112(mat(112, 112, [&](int c, int k) { return at(qk, c, k); })), 0));
    op.push_back(hi_lo(frag112(mat(112, 112, [&](int c, int k) { return at(vo, k, c); })), 0));
    op.push_back(hi_lo(frag112(mat(112, 112, [&](int c, int k) { return at(vo, c, k); })), 0));
  }
  auto F = [&](const std::vector<double> &v, int ld, int r, int c) { return v[(size_t)r * ld + c]; };
  // the fitting operands in MFMA fragment order: the 16 x 32 fragment (column tile t,
  // k step s) is 64 lanes x 8 contiguous values, lane l holding row 16 t + l % 16,
  // k = 32 s + 8 (l / 16) .. + 8; so one wave's fragment load is 1 KB of whole lines
  auto frag = [](const std::vector<float> &v, int R, int K) {
    std::vector<float> o(v.size());
    const int S = K / 32;
    for (int t = 0; t < R / 16; ++t)
      for (int st = 0; st < S; ++st)
        for (int l = 0; l < 64; ++l)
          for (int e = 0; e < 8; ++e)
            o[(((size_t)t * S + st) * 64 + l) * 8 + e] = v[(size_t)(16 * t + l % 16) * K + 32 * st + 8 * (l / 16) + e];
    return o;
  };
  for (int hd = 0; hd < h.nheads; ++hd) {
    const auto f1t = mat(FH, ND, [&](int c, int k) { return F(h.F1[hd], FH, k, c); });
    const auto f1 = mat(ND, 256, [&](int c, int k) { return k < FH ? F(h.F1[hd], FH, c, k) : 0.0; });
    const auto f2t = mat(FH, 256, [&](int c, int k) { return k < FH ? F(h.F2[hd], FH, k, c) : 0.0; });
    const auto f2 = mat(FH, 256, [&](int c, int k) { return k < FH ? F(h.F2[hd], FH, c, k) : 0.0; });
    const auto f3t = mat(FH, 256, [&](int c, int k) { return k < FH ? F(h.F3[hd], FH, k, c) : 0.0; });
    const auto f3 = mat(FH, 256, [&](int c, int k) { return k < FH ? F(h.F3[hd], FH, c, k) : 0.0; });
    const std::vector<float> fr[] = {frag(f1t, FH, ND), frag(f1, ND, 256), frag(f2t, FH, 256),
                                     frag(f2, FH, 256), frag(f3t, FH, 256), frag(f3, FH, 256)};
    for (const auto &v : fr) {
      op.push_back(hi_lo(v, 0));
      op.push_back(hi_lo(v, 1));
    }
  }
}

// Points the structures at a weight image based at `base` (a device address, or any
// placeholder for the host-side check).
void bind_image(const Image &im, int pr, const unsigned char *base, Weights<float> &w, WeightsB16 &wp) {
  w = Weights<float>{};
  wp = WeightsB16{};
  size_t k = 0;
  auto F = [&]() { return (const float *)(base + im.tab[k++]); };
  w.w1s = F(); w.Bt = F(); w.b2 = F(); w.b3 = F();
  for (int a = 0; a < NATTN; ++a) {
    w.gamma[a] = F(); w.beta[a] = F();
  }
  w.nheads = im.nheads;
  for (int hd = 0; hd < im.nheads; ++hd) {
    w.c1[hd] = F(); w.c2[hd] = F(); w.c3[hd] = F(); w.F4[hd] = F();
    w.F4d[hd] = (const double *)(base + im.tab[k++]);
    w.ebias[hd] = (const double *)(base + im.tab[k++]);
    w.c4[hd] = im.c4[hd];
    w.hw[hd] = hd == 0 ? 1.0 : 0.0;  // head 0 alone until dp_set_head_weights
  }
  if (pr == DP_FP32) {
    k = 0;
    auto P = [&]() { return (const float *)(base + im.f32[k++]); };
    w.W2T = P(); w.W2 = P(); w.W3T = P(); w.W3 = P();
    for (int a = 0; a < NATTN; ++a) {
      w.WqkT[a] = P(); w.Wqk[a] = P(); w.WvoT[a] = P(); w.Wvo[a] = P();
    }
    for (int hd = 0; hd < im.nheads; ++hd) {
      w.F1T[hd] = P(); w.F1[hd] = P(); w.F2T[hd] = P(); w.F2[hd] = P(); w.F3T[hd] = P(); w.F3[hd] = P();
    }
  } else {
    k = 0;
    auto P = [&]() { return (const bf16_t *)(base + im.b16[k++]); };
    wp.W2T = P(); wp.W3T = P(); wp.W3 = P(); wp.W2 = P();
    for (int a = 0; a < NATTN; ++a) {
      wp.WqkT[a] = P(); wp.Wqk[a] = P(); wp.WvoT[a] = P(); wp.Wvo[a] = P();
    }
    for (int hd = 0; hd < im.nheads; ++hd) {
      for (int x = 0; x < 2; ++x) { wp.F1T[hd][x] = P(); }
      for (int x = 0; x < 2; ++x) { wp.F1[hd][x] = P(); }
      for (int x = 0; x < 2; ++x) { wp.F2T[hd][x] = P(); }
      for (int x = 0; x < 2; ++x) { wp.F2[hd][x] = P(); }
      for (int x = 0; x < 2; ++x) { wp.F3T[hd][x] = P(); }
      for (int x = 0; x < 2; ++x) { wp.F3[hd][x] = P(); }
    }
  }
}

// The weight pointers the kernels of precision `pr` read, by name.
std::vector<std::pair<std::string, const void **>> weight_fields(int pr, Weights<float> &w, WeightsB16 &wp) {
  std::vector<std::pair<std::string, const void **>> f;
  auto add = [&](const std::string &name, const void *member) { f.emplace_back(name, (const void **)member); };
  add("w1s", &w.w1s); add("Bt", &w.Bt); add("b2", &w.b2); add("b3", &w.b3);
  for (int a = 0; a < NATTN; ++a) {
    add("gamma" + std::to_string(a), &w.gamma[a]);
    add("beta" + std::to_string(a), &w.beta[a]);
  }
  for (int hd = 0; hd < w.nheads; ++hd) {
    const std::string t = hd ? "." + std::to_string(hd) : "";
    add("c1" + t, &w.c1[hd]); add("c2" + t, &w.c2[hd]); add("c3" + t, &w.c3[hd]); add("F4" + t, &w.F4[hd]);
    add("F4d" + t, &w.F4d[hd]); add("ebias" + t, &w.ebias[hd]);
  }
  if (pr == DP_FP32) {
    add("W2T", &w.W2T); add("W2", &w.W2); add("W3T", &w.W3T); add("W3", &w.W3);
    for (int a = 0; a < NATTN; ++a) {
      const std::string t = std::to_string(a);
      add("WqkT" + t, &w.WqkT[a]); add("Wqk" + t, &w.Wqk[a]); add("WvoT" + t, &w.WvoT[a]); add("Wvo" + t, &w.Wvo[a]);
    }
    for (int hd = 0; hd < w.nheads; ++hd) {
      const std::string t = hd ? "." + std::to_string(hd) : "";
      add("F1T" + t, &w.F1T[hd]); add("F1" + t, &w.F1[hd]); add("F2T" + t, &w.F2T[hd]); add("F2" + t, &w.F2[hd]);
      add("F3T" + t, &w.F3T[hd]); add("F3" + t, &w.F3[hd]);
    }
    return f;
  }
  add("b16.W2T", &wp.W2T); add("b16.W3T", &wp.W3T); add("b16.W3", &wp.W3); add("b16.W2", &wp.W2);
  for (int a = 0; a < NATTN; ++a) {
    const std::string t = std::to_string(a);
    add("b16.WqkT" + t, &wp.WqkT[a]); add("b16.Wqk" + t, &wp.Wqk[a]);
    add("b16.WvoT" + t, &wp.WvoT[a]); add("b16.Wvo" + t, &wp.Wvo[a]);
  }
  for (int hd = 0; hd < w.nheads; ++hd)
    for (int x = 0; x < 2; ++x) {
      const std::string t = (hd ? "." + std::to_string(hd) : "") + (x ? ".lo" : ".hi");
      add("b16.F1T" + t, &wp.F1T[hd][x]); add("b16.F1" + t, &wp.F1[hd][x]); add("b16.F2T" + t, &wp.F2T[hd][x]);
      add("b16.F2" + t, &wp.F2[hd][x]); add("b16.F3T" + t, &wp.F3T[hd][x]); add("b16.F3" + t, &wp.F3[hd][x]);
    }
  return f;
}

// Every pointer the kernels of precision `pr` read lies inside the image [base, base + bytes).
// A member left unbound (null) or pointing elsewhere is reported by name.
bool check_bound(int pr, const unsigned char *base, size_t bytes, Weights<float> &w, WeightsB16 &wp,
                 std::string &why) {
  for (const auto &f : weight_fields(pr, w, wp)) {
    const unsigned char *c = (const unsigned char *)*f.second;
    if (!c || c < base || c >= base + bytes) {
      why = "weight pointer " + f.first + (c ? " outside the weight image" : " is null");
      return false;
    }
  }
  return true;
}

int build_weights(dp_model *m, const HostModel &h) {
  Image im;
  pack_weights(h, m->prec, im);
  HIP_TRY(hipMalloc(&m->wbuf, im.pk.bytes.size()));
  HIP_TRY(hipMemcpy(m->wbuf, im.pk.bytes.data(), im.pk.bytes.size(), hipMemcpyHostToDevice));
  const unsigned char *base = (const unsigned char *)m->wbuf;
  bind_image(im, m->prec, base, m->wf, m->wp);
  std::string why;
  if (!check_bound(m->prec, base, im.pk.bytes.size(), m->wf, m->wp, why)) {
    set_error("dp_model_load: " + why);
    return DP_ERR_MODEL_FILE;
  }
  return DP_OK;
}

}  // namespace

void free_ws(Workspace &ws) {
  void *ps[] = {ws.cell_of, ws.cell_count, ws.cell_start, ws.cell_cursor, ws.cell_atoms, ws.nlist, ws.nnei, ws.done,
                ws.Gsave, ws.Tsave, ws.D, ws.Ei, ws.Eh, ws.Ehsys, ws.g, ws.vpart, ws.red, ws.grids, ws.sys_off, ws.sys_of, ws.slist,
                ws.snnei, ws.xref, ws.flags, ws.gE, ws.bidx, ws.bcnt};
  for (void *p : ps)
    if (p) (void)hipFree(p);
  void *hs[] = {ws.flags_host, ws.grids_host, ws.off_host};
  for (void *p : hs)
    if (p) (void)hipHostFree(p);
  if (ws.side) (void)hipStreamDestroy(ws.side);
  if (ws.fork_ev) (void)hipEventDestroy(ws.fork_ev);
  if (ws.join_ev) (void)hipEventDestroy(ws.join_ev);
  ws = Workspace{};
}

// Device bytes the workspace holds per atom (the serving admission model uses it).
size_t ws_bytes_per_atom(int prec) {
  size_t b = 4 * sizeof(int)                              // cell_of, cell_atoms, nnei, sys_of
             + (size_t)SEL * sizeof(int)                  // nlist
             + (size_t)M * 4 * sizeof(float)              // Tsave
             + (size_t)ND * sizeof(float)                 // D
             + (1 + MAXH) * sizeof(double)                // Ei, Eh
             + (size_t)SEL * sizeof(float4)               // g
             + 9 * sizeof(double)                         // vpart
             + 2 * sizeof(int);                           // backward atom lists
  b += (size_t)NATTN * GSAVE_LAYER * sizeof(float);  // Gsave
  return b;
}

int ensure_ws(Workspace &ws, int prec, int64_t n, int nsys, bool skin, bool lists_only) {
  if (!ws.flags) {
    HIP_TRY(hipMalloc(&ws.flags, 4 * sizeof(unsigned)));
    HIP_TRY(hipHostMalloc(&ws.flags_host, 4 * sizeof(unsigned), hipHostMallocDefault));
    HIP_TRY(hipMalloc(&ws.cell_count, (MAX_CELLS + 1) * sizeof(int)));
    HIP_TRY(hipMalloc(&ws.cell_start, (MAX_CELLS + 1) * sizeof(int)));
    HIP_TRY(hipMalloc(&ws.cell_cursor, MAX_CELLS * sizeof(int)));
    HIP_TRY(hipMalloc(&ws.red, 64 * sizeof(double)));
    HIP_TRY(hipMalloc(&ws.gE, sizeof(double)));
    HIP_TRY(hipMalloc(&ws.bcnt, 2 * sizeof(int)));
    HIP_TRY(hipStreamCreateWithFlags(&ws.side, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&ws.fork_ev, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&ws.join_ev, hipEventDisableTiming));
  }
  if (nsys > ws.cap_sys) {
    const int cs = std::max(nsys, 8);
    if (ws.grids) (void)hipFree(ws.grids);
    if (ws.sys_off) (void)hipFree(ws.sys_off);
    if (ws.done) (void)hipFree(ws.done);
    if (ws.Ehsys) (void)hipFree(ws.Ehsys);
    if (ws.grids_host) (void)hipHostFree(ws.grids_host);
    if (ws.off_host) (void)hipHostFree(ws.off_host);
    ws.grids = nullptr; ws.sys_off = nullptr; ws.done = nullptr; ws.Ehsys = nullptr; ws.grids_host = nullptr;
    ws.off_host = nullptr;
    ws.cap_sys = 0;
    HIP_TRY(hipMalloc(&ws.grids, cs * sizeof(Grid)));
    HIP_TRY(hipMalloc(&ws.sys_off, (cs + 1) * sizeof(int)));  // cs >= 8: [2..3] also hold a centre range
    HIP_TRY(hipMalloc(&ws.done, (2 * cs + 1) * sizeof(int)));
    HIP_TRY(hipMalloc(&ws.Ehsys, (size_t)cs * MAXH * sizeof(double)));
    HIP_TRY(hipHostMalloc(&ws.grids_host, cs * sizeof(Grid), hipHostMallocDefault));
    HIP_TRY(hipHostMalloc(&ws.off_host, (cs + 1) * sizeof(int), hipHostMallocDefault));
    ws.cap_sys = cs;
    ws.gen += 1;
  }
  if (n > ws.cap) {
    const int64_t cap = std::max<int64_t>(n, ws.cap + ws.cap / 4);
    void *ps[] = {ws.cell_of, ws.cell_atoms, ws.nlist, ws.nnei, ws.Gsave, ws.Tsave, ws.D, ws.Ei, ws.Eh, ws.g,
                  ws.vpart, ws.sys_of, ws.slist, ws.snnei, ws.xref, ws.bidx};
    for (void *p : ps)
      if (p) (void)hipFree(p);
    ws.cell_of = ws.cell_atoms = ws.nlist = ws.nnei = ws.sys_of = ws.slist = ws.snnei = ws.bidx = nullptr;
    ws.Gsave = ws.Tsave = ws.D = nullptr;
    ws.Ei = ws.Eh = ws.vpart = ws.xref = nullptr;
    ws.g = nullptr;
    ws.cap = 0;
    HIP_TRY(hipMalloc(&ws.cell_of, cap * sizeof(int)));
    HIP_TRY(hipMalloc(&ws.cell_atoms, cap * sizeof(int)));
    HIP_TRY(hipMalloc(&ws.sys_of, cap * sizeof(int)));
    HIP_TRY(hipMalloc(&ws.nlist, cap * SEL * sizeof(int)));
    HIP_TRY(hipMalloc(&ws.nnei, cap * sizeof(int)));
    if (!lists_only) {  // the attention descriptor's buffers
      HIP_TRY(hipMalloc(&ws.Gsave, cap * (size_t)NATTN * GSAVE_LAYER * sizeof(float)));
      HIP_TRY(hipMalloc(&ws.Tsave, cap * (size_t)M * 4 * sizeof(float)));
      HIP_TRY(hipMalloc(&ws.bidx, 2 * cap * sizeof(int)));
      HIP_TRY(hipMalloc(&ws.D, (cap + 16) * (size_t)ND * sizeof(float)));  // 16 spare rows for batched readers
      HIP_TRY(hipMemset(ws.D, 0, (cap + 16) * (size_t)ND * sizeof(float)));
      HIP_TRY(hipMalloc(&ws.Eh, cap * MAXH * sizeof(double)));
    }
    HIP_TRY(hipMalloc(&ws.Ei, cap * sizeof(double)));
    HIP_TRY(hipMalloc(&ws.g, cap * (size_t)SEL * sizeof(float4)));
    HIP_TRY(hipMalloc(&ws.vpart, cap * 9 * sizeof(double)));
    ws.cap = cap;
    ws.skin_cap = 0;
    ws.gen += 1;
  }
  if (skin && ws.skin_cap < ws.cap) {
    void *ps[] = {ws.slist, ws.snnei, ws.xref};
    for (void *p : ps)
      if (p) (void)hipFree(p);
    ws.slist = ws.snnei = nullptr;
    ws.xref = nullptr;
    HIP_TRY(hipMalloc(&ws.slist, ws.cap * (size_t)SKIN_CAP * sizeof(int)));
    HIP_TRY(hipMalloc(&ws.snnei, ws.cap * sizeof(int)));
    HIP_TRY(hipMalloc(&ws.xref, ws.cap * 3 * sizeof(double)));
    ws.skin_cap = ws.cap;
    ws.gen += 1;
  }
  return DP_OK;
}

// ------------------------------------------------------------ allocation-free step
// Workspace of dp_compute_device_noalloc: one file-scope device array per GPU, held
// until the process ends.  Host code never passes `scratch` itself to a kernel (in host
// code the name is only a stand-in); it passes the device address hipGetSymbolAddress
// returns for the current device, kept per device in g_noalloc.
constexpr size_t NOALLOC_BYTES = (size_t)128 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

// Points a workspace for `cap` atoms (one system) at consecutive 256-byte aligned pieces
// from `base`; returns the bytes used.  base == nullptr only measures.
size_t carve_ws(Workspace &ws, unsigned char *base, int64_t cap) {
  size_t off = 0;
  auto take = [&](auto *&p, size_t bytes) {
    off = (off + 255) & ~size_t(255);
    p = reinterpret_cast<std::remove_reference_t<decltype(p)>>(base ? base + off : nullptr);
    off += bytes;
  };
  const size_t c = (size_t)cap;
  take(ws.flags, 4 * sizeof(unsigned));
  take(ws.cell_count, (MAX_CELLS + 1) * sizeof(int));
  take(ws.cell_start, (MAX_CELLS + 1) * sizeof(int));
  take(ws.cell_cursor, MAX_CELLS * sizeof(int));
  take(ws.red, 64 * sizeof(double));
  take(ws.gE, sizeof(double));
  take(ws.bcnt, 2 * sizeof(int));
  take(ws.grids, sizeof(Grid));
  take(ws.sys_off, 4 * sizeof(int));
  take(ws.done, 3 * sizeof(int));
  take(ws.sys_of, c * sizeof(int));
  take(ws.cell_of, c * sizeof(int));
  take(ws.cell_atoms, c * sizeof(int));
  take(ws.nlist, c * SEL * sizeof(int));
  take(ws.nnei, c * sizeof(int));
  take(ws.Gsave, c * NATTN * GSAVE_LAYER * sizeof(float));
  take(ws.Tsave, c * M * 4 * sizeof(float));
  take(ws.bidx, 2 * c * sizeof(int));
  take(ws.D, (c + 16) * ND * sizeof(float));
  take(ws.Ei, c * sizeof(double));
  take(ws.Eh, c * MAXH * sizeof(double));
  take(ws.Ehsys, MAXH * sizeof(double));
  take(ws.g, c * SEL * sizeof(float4));
  take(ws.vpart, c * 9 * sizeof(double));
  ws.cap = cap;
  ws.cap_sys = 1;
  return off;
}

struct NoAllocDevice {
  bool ready = false;
  Workspace ws;  // device pieces inside `scratch`; pinned staging, side stream and events made at set-up
};
constexpr int NOALLOC_MAX_DEVICES = 64;
NoAllocDevice g_noalloc[NOALLOC_MAX_DEVICES];
std::mutex g_noalloc_mu;

// Once per device, with that device current (called by dp_model_load): the device
// address of `scratch`, the workspace carved from it, and the host-side objects the step
// needs (pinned staging, the side stream and events of the bf16 backward).
int noalloc_setup(int device) {
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (device < 0 || device >= NOALLOC_MAX_DEVICES) return DP_OK;  // entry point then reports it
  NoAllocDevice &d = g_noalloc[device];
  if (d.ready) return DP_OK;
  void *ptr = nullptr;
  HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  Workspace ws;
  if (carve_ws(ws, (unsigned char *)ptr, DP_NOALLOC_MAX_ATOMS) > NOALLOC_BYTES) {
    set_error("allocation-free workspace: layout exceeds the static array");
    return DP_ERR_HIP;
  }
  HIP_TRY(hipHostMalloc(&ws.flags_host, 4 * sizeof(unsigned), hipHostMallocDefault));
  HIP_TRY(hipHostMalloc(&ws.grids_host, sizeof(Grid), hipHostMallocDefault));
  HIP_TRY(hipHostMalloc(&ws.off_host, 4 * sizeof(int), hipHostMallocDefault));
  HIP_TRY(hipStreamCreateWithFlags(&ws.side, hipStreamNonBlocking));
  HIP_TRY(hipEventCreateWithFlags(&ws.fork_ev, hipEventDisableTiming));
  HIP_TRY(hipEventCreateWithFlags(&ws.join_ev, hipEventDisableTiming));
  d.ws = ws;
  d.ready = true;
  return DP_OK;
}

constexpr int64_t MAX_ATOMS = 1 << 24;

// Validates a box and fills the cell grid for cells of edge >= cutoff.  box == NULL:
// open boundaries (the grid is then built on the device from the coordinates).
int make_grid(double rc, double cutoff, const double *box, Grid &g) {
  std::memset(&g, 0, sizeof(g));
  if (!box) return DP_OK;
  for (int k = 0; k < 9; ++k)
    if (!std::isfinite(box[k])) {
      set_error("box has a non-finite entry");
      return DP_ERR_NONFINITE;
    }
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      if (a != b && box[3 * a + b] != 0.0) {
        set_error("box must be orthorhombic (off-diagonal entries exactly 0)");
        return DP_ERR_BOX;
      }
  g.periodic = 1;
  int nct = 1;
  for (int a = 0; a < 3; ++a) {
    const double L = box[4 * a];
    if (!(L >= 2.0 * rc)) {
      set_error("every box edge must be at least 2 rc");
      return DP_ERR_BOX;
    }
    if (!(L >= 2.0 * cutoff)) return DP_ERR_BOX;  // only for the skin cutoff: caller falls back
    int nc = (int)std::floor(L / (cutoff * (1.0 + 1e-9)));
    nc = std::max(1, std::min(nc, MAX_CELLS_PER_DIM));
    g.L[a] = L;
    g.invL[a] = 1.0 / L;
    g.nc[a] = nc;
    g.cw[a] = L / nc;
    g.icw[a] = nc / L;
    nct *= nc;
  }
  g.ncells = nct;
  return DP_OK;
}

namespace {

int flags_status(unsigned f) {
  if (f & FLAG_NONFINITE) { set_error("non-finite coordinate"); return DP_ERR_NONFINITE; }
  if (f & FLAG_TYPE) { set_error("atom type outside [0, ntypes)"); return DP_ERR_TYPE; }
  if (f & FLAG_OVERLAP) { set_error("two atoms at distance 0"); return DP_ERR_OVERLAP; }
  if (f & FLAG_TOO_DENSE) { set_error("more than DP_MAX_CANDIDATES neighbours within rc"); return DP_ERR_TOO_LARGE; }
  if (f & FLAG_INCOMPLETE) {
    set_error("an atom has more than sel neighbours within rc; the message-passing models need complete lists");
    return DP_ERR_TOO_LARGE;
  }
  return DP_OK;
}

// Event k is recorded before phase k (k = 0..5) and after the last phase.
void mark(dp_model *m, int k, hipStream_t st) {
  if (m->prof) (void)hipEventRecord(m->ev[k], st);
}
void collect(dp_model *m, int last) {
  if (!m->prof) return;
  for (int k = 0; k < last; ++k) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, m->ev[k], m->ev[k + 1]) == hipSuccess) {
      m->prof_ms[k] += ms;
      m->prof_calls[k] += 1;
    }
  }
}

}  // namespace

// Enqueues one step (no host synchronisation; nothing here allocates).  The per-system
// grids and atom offsets must already be in ws.grids_host / ws.off_host; they are
// copied to the device first unless `open_single` (one open system, grid built on the
// device).  Outputs are written only if the step raised no error flag.
int enqueue_step(dp_model *m, Workspace &ws, const StepArgs &a, hipStream_t st, bool profile) {
  dp_model *pm = profile ? m : nullptr;
  const int n = (int)a.n;
  // centres: every atom, or (one system with ghost atoms) the first n_centres
  const int nc = (a.nsys == 1 && a.n_centres >= 0 && a.n_centres < a.n) ? (int)a.n_centres : n;
  // this call's part of them: all, or one chunk c0 .. c1-1 of a single system
  const int cb = a.nsys == 1 ? (int)a.c0 : 0;
  const int ce = (a.nsys == 1 && a.c1 >= 0) ? (int)a.c1 : nc;
  if (a.first_chunk) {
    if (!a.open_single)
      HIP_TRY(hipMemcpyAsync(ws.grids, ws.grids_host, a.nsys * sizeof(Grid), hipMemcpyHostToDevice, st));
    if (nc < n) {  // off_host[2..3]: the centre range, reduced for the energy
      ws.off_host[2] = 0;
      ws.off_host[3] = nc;
    }
    HIP_TRY(hipMemcpyAsync(ws.sys_off, ws.off_host, (nc < n ? 4 : a.nsys + 1) * sizeof(int), hipMemcpyHostToDevice,
                           st));
    launch_prologue(ws, a.nsys, n, a.lists == LISTS_SKIN_REUSE ? 0 : a.ncells + 1, true, st);
  } else {
    launch_prologue(ws, a.nsys, 0, 0, false, st);  // a later chunk: only the backward's atom lists restart
  }
  if (pm) mark(pm, 0, st);
  switch (a.lists) {
    case LISTS_FRESH:
      if (a.first_chunk) launch_cells(ws, a.X, a.types, n, m->ntypes, a.open_single, a.ncells, m->rc, st);
      if (nc < n)
        launch_nlist(ws, a.X, n, 0, n, nc, m->rc, false, st);  // ghosts get empty lists
      else
        launch_nlist(ws, a.X, n, cb, ce, n, m->rc, false, st);
      break;
    case LISTS_SKIN_BUILD:
      launch_cells(ws, a.X, a.types, n, m->ntypes, a.open_single, a.ncells, m->rc + m->skin, st);
      launch_nlist(ws, a.X, n, 0, n, n, m->rc + m->skin, true, st);
      launch_skin_ref(ws, a.X, n, st);
      launch_filter(ws, a.X, n, m->rc, st);
      break;
    case LISTS_SKIN_REUSE: {
      const double h = 0.5 * m->skin * (1.0 - 1e-9);
      launch_skin_check(ws, a.X, a.types, n, m->ntypes, h * h, st);
      launch_filter(ws, a.X, n, m->rc, st);
      break;
    }
  }
  HIP_TRY(hipGetLastError());
  const float rc = (float)m->rc, rcs = (float)m->rcs, eps = (float)m->ln_eps;
  const bool bwd = a.forces || a.virial;
  if (pm) mark(pm, 1, st);
  if (m->prec == DP_BF16)
    launch_descriptor_fwd_b16(m->wf, m->wp, ws, a.X, a.types, n, cb, ce, rc, rcs, eps, st);
  else
    launch_descriptor_fwd<float>(m->wf, ws, a.X, a.types, n, cb, ce, rc, rcs, eps, st);
  if (pm) mark(pm, 2, st);
  if (m->prec == DP_BF16)
    launch_fitting_b16(m->wf, m->wp, ws, a.types, cb, ce, bwd, st);
  else
    launch_fitting<float>(m->wf, ws, a.types, cb, ce, bwd, st);
  if (pm) mark(pm, 3, st);
  // energies over the centre atoms (every atom, or the first nc of one system with ghosts)
  const int *eoff = nc < n ? ws.sys_off + 2 : ws.sys_off;
  if (!bwd && a.last_chunk) launch_reduce(ws, eoff, a.nsys, a.energy, a.atom_energy, nullptr, m->wf.nheads, st);
  if (pm) mark(pm, 4, st);
  if (bwd) {
    if (m->prec == DP_BF16)
      launch_descriptor_bwd_b16(m->wf, m->wp, ws, a.X, a.types, n, cb, ce, rc, rcs, eps, st);
    else
      launch_descriptor_bwd<float>(m->wf, ws, a.X, a.types, n, cb, ce, rc, rcs, eps, st);
    if (pm) mark(pm, 5, st);
    if (a.last_chunk) {
      double *F = a.forces;
      if (!F) F = (double *)ws.D;  // forces not requested: park them in the (now free) descriptor buffer
      launch_forces(ws, a.X, n, nullptr, F, a.lists == LISTS_SKIN_REUSE, nc < n, st);
      launch_reduce(ws, eoff, a.nsys, a.energy, a.atom_energy, a.virial, m->wf.nheads, st);
    }
    if (pm) mark(pm, 6, st);
  }
  HIP_TRY(hipGetLastError());
  return DP_OK;
}

// Status of a finished step from the flag words copied to ws.flags_host.
int step_status(const Workspace &ws) {
  const unsigned f = ws.flags_host[0];
  const int s = flags_status(f);
  if (s != DP_OK) return s;
  if (f & (FLAG_STALE | FLAG_SKIN_FULL)) return DP_RETRY;
  return ws.flags_host[1] ? DP_WARN_SEL_OVERFLOW : DP_OK;
}

namespace {

bool same_bits(const double *a, const double *b, int n) { return std::memcmp(a, b, n * sizeof(double)) == 0; }

// One step of a single system through a captured graph: captured on first use of a
// configuration (list mode, sizes, pointers, box, stream), replayed afterwards.
int launch_graph(dp_model *m, const StepArgs &a, hipStream_t st) {
  GraphKey k{};
  k.lists = a.lists;
  k.n = a.n;
  k.X = a.X; k.types = a.types; k.energy = a.energy; k.forces = a.forces; k.virial = a.virial;
  k.atom_energy = a.atom_energy;
  k.stream = st;
  k.open_single = a.open_single;
  if (!a.open_single) std::memcpy(k.box, m->ws.grids_host[0].L, 3 * sizeof(double));
  k.ws_gen = m->ws.gen;
  // graphs captured on an earlier workspace point at freed buffers: drop them
  for (auto &e : m->graphs)
    if (e.exec && e.key.ws_gen != k.ws_gen) {
      (void)hipGraphExecDestroy(e.exec);
      e.exec = nullptr;
    }
  for (auto &e : m->graphs)
    if (e.exec && std::memcmp(&e.key, &k, sizeof(k)) == 0) {
      // the host-side grid table is uploaded outside the graph (same values as at capture)
      if (!a.open_single)
        HIP_TRY(hipMemcpyAsync(m->ws.grids, m->ws.grids_host, sizeof(Grid), hipMemcpyHostToDevice, st));
      HIP_TRY(hipGraphLaunch(e.exec, st));
      return DP_OK;
    }
  GraphEntry &slot = m->graphs[m->graph_next];
  m->graph_next = (m->graph_next + 1) % (int)(sizeof(m->graphs) / sizeof(m->graphs[0]));
  if (slot.exec) (void)hipGraphExecDestroy(slot.exec);
  slot.exec = nullptr;
  hipGraph_t graph = nullptr;
  HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  int s = enqueue_step(m, m->ws, a, st, false);
  const hipError_t e = hipStreamEndCapture(st, &graph);
  if (s != DP_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return s;
  }
  HIP_TRY(e);
  const hipError_t ei = hipGraphInstantiate(&slot.exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  HIP_TRY(ei);
  slot.key = k;
  HIP_TRY(hipGraphLaunch(slot.exec, st));
  return DP_OK;
}

// One step of one system: list mode from the skin state, eager or graph launch, the
// flag words read back, and a redo with fresh lists when the skin list was stale.
int run_single(dp_model *m, StepArgs a, const double *box, hipStream_t st) {
  Workspace &ws = m->ws;
  Grid g, gs;
  int s = make_grid(m->rc, m->rc, box, g);
  if (s != DP_OK) return s;
  bool skin = m->skin > 0.0;
  if (skin && box) skin = make_grid(m->rc, m->rc + m->skin, box, gs) == DP_OK;
  a.open_single = box == nullptr;
  a.nsys = 1;
  s = ensure_ws(ws, m->prec, a.n, 1, skin);
  if (s != DP_OK) return s;
  ws.off_host[0] = 0;
  ws.off_host[1] = (int)a.n;
  if (skin) {
    const bool same = m->skin_valid && m->skin_n == a.n && m->skin_open == a.open_single &&
                      (a.open_single || same_bits(m->skin_box, box, 9));
    a.lists = (same && m->skin_age < m->rebuild_every) ? LISTS_SKIN_REUSE : LISTS_SKIN_BUILD;
  } else {
    a.lists = LISTS_FRESH;
  }
  // the legacy default stream cannot be captured: a graph then runs on the model's own
  // stream, ordered after the work already queued on the default stream
  const bool graph = m->use_graph && !m->prof;
  if (graph && st == nullptr) {
    HIP_TRY(hipEventRecord(m->dep_ev, nullptr));
    st = m->own_stream;
    HIP_TRY(hipStreamWaitEvent(st, m->dep_ev, 0));
  }
  for (int attempt = 0; attempt < 3; ++attempt) {
    const bool skin_cells = a.lists != LISTS_FRESH;
    ws.grids_host[0] = skin_cells && !a.open_single ? gs : g;
    a.ncells = a.open_single ? MAX_CELLS : ws.grids_host[0].ncells;
    if (graph) {
      s = launch_graph(m, a, st);
    } else if (m->chunk > 0 && a.lists == LISTS_FRESH && a.n > m->chunk) {
      // the centres in chunks of m->chunk atoms, each chunk a sequence of launches
      for (int64_t c0 = 0; c0 < a.n && s == DP_OK; c0 += m->chunk) {
        StepArgs c = a;
        c.c0 = c0;
        c.c1 = std::min<int64_t>(a.n, c0 + m->chunk);
        c.first_chunk = c0 == 0;
        c.last_chunk = c.c1 == a.n;
        s = enqueue_step(m, ws, c, st, false);
      }
    } else {
      s = enqueue_step(m, ws, a, st, m->prof);
    }
    if (s != DP_OK) return s;
    HIP_TRY(hipMemcpyAsync(ws.flags_host, ws.flags, 4 * sizeof(unsigned), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    s = step_status(ws);
    if (s == DP_RETRY) {
      m->skin_valid = false;
      // stale skin list: rebuild it; a full skin row: fresh lists for this step
      a.lists = (a.lists == LISTS_SKIN_REUSE) ? LISTS_SKIN_BUILD : LISTS_FRESH;
      m->skin_rebuilds_forced += 1;
      continue;
    }
    if (s < 0) {
      m->skin_valid = false;
      return s;
    }
    if (!graph) collect(m, (a.forces || a.virial) ? 6 : 4);
    m->fwd_lists = a.lists;
    if (a.lists == LISTS_SKIN_BUILD) {
      m->skin_valid = true;
      m->skin_age = 1;
      m->skin_n = a.n;
      m->skin_open = a.open_single;
      if (box) std::memcpy(m->skin_box, box, 9 * sizeof(double));
      m->skin_builds += 1;
    } else if (a.lists == LISTS_SKIN_REUSE) {
      m->skin_age += 1;
    }
    return s;
  }
  set_error("neighbour lists could not be rebuilt");
  return DP_ERR_HIP;
}

}  // namespace
}  // namespace dp

using namespace dp;

extern "C" {

const char *dp_status_string(int s) {
  switch (s) {
    case DP_OK: return "ok";
    case DP_WARN_SEL_OVERFLOW: return "warning: neighbour list truncated to sel";
    case DP_ERR_ARG: return "invalid argument";
    case DP_ERR_MODEL_FILE: return "bad model file";
    case DP_ERR_TYPE: return "atom type out of range";
    case DP_ERR_BOX: return "unsupported box";
    case DP_ERR_OVERLAP: return "overlapping atoms";
    case DP_ERR_NONFINITE: return "non-finite input";
    case DP_ERR_OOM: return "device out of memory";
    case DP_ERR_TOO_LARGE: return "system too large or too dense";
    case DP_ERR_HIP: return "HIP runtime error";
    case DP_ERR_TIMEOUT: return "timeout";
    default: return "unknown status";
  }
}

const char *dp_last_error(void) { return g_last_error.c_str(); }

int dp_model_load(const char *path, int precision, int device, dp_model **out) {
  g_last_error.clear();
  if (!path || !out || (precision != DP_FP32 && precision != DP_BF16)) {
    set_error("dp_model_load: bad argument");
    return DP_ERR_ARG;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    set_error("dp_model_load: no such HIP device");
    return DP_ERR_ARG;
  }
  HostModel h;
  int s = read_model(path, h);
  if (s != DP_OK) return s;
  HIP_TRY(hipSetDevice(device));
  dp_model *m = new dp_model();
  m->device = device;
  m->prec = precision;
  m->rc = h.rc;
  m->rcs = h.rcs;
  m->ln_eps = h.eps;
  m->sel = h.sel;
  m->ntypes = h.ntypes;
  s = build_weights(m, h);
  if (s == DP_OK) s = noalloc_setup(device);
  if (s == DP_OK && (hipStreamCreateWithFlags(&m->own_stream, hipStreamNonBlocking) != hipSuccess ||
                     hipEventCreateWithFlags(&m->dep_ev, hipEventDisableTiming) != hipSuccess)) {
    set_error("dp_model_load: stream creation failed");
    s = DP_ERR_HIP;
  }
  if (s != DP_OK) {
    dp_model_free(m);
    return s;
  }
  *out = m;
  return DP_OK;
}

void dp_model_free(dp_model *m) {
  if (!m) return;
  (void)hipSetDevice(m->device);
  (void)hipDeviceSynchronize();
  for (int k = 0; k < 8; ++k)
    if (m->ev[k]) (void)hipEventDestroy(m->ev[k]);
  for (auto &e : m->graphs)
    if (e.exec) (void)hipGraphExecDestroy(e.exec);
  if (m->own_stream) (void)hipStreamDestroy(m->own_stream);
  if (m->dep_ev) (void)hipEventDestroy(m->dep_ev);
  free_ws(m->ws);
  if (m->wbuf) (void)hipFree(m->wbuf);
  delete m;
}

int dp_check_model_file(const char *path, int precision, const char *unbind, size_t *image_bytes) {
  g_last_error.clear();
  if (!path || (precision != DP_FP32 && precision != DP_BF16)) {
    set_error("dp_check_model_file: bad argument");
    return DP_ERR_ARG;
  }
  HostModel h;
  int s = read_model(path, h);
  if (s != DP_OK) return s;
  Image im;
  pack_weights(h, precision, im);
  const unsigned char *base = im.pk.bytes.data();
  Weights<float> w;
  WeightsB16 wp;
  bind_image(im, precision, base, w, wp);
  if (unbind) {
    bool found = false;
    for (const auto &f : weight_fields(precision, w, wp))
      if (f.first == unbind) {
        *f.second = nullptr;
        found = true;
      }
    if (!found) {
      set_error(std::string("dp_check_model_file: no weight named ") + unbind);
      return DP_ERR_ARG;
    }
  }
  if (image_bytes) *image_bytes = im.pk.bytes.size();
  std::string why;
  if (!check_bound(precision, base, im.pk.bytes.size(), w, wp, why)) {
    set_error("dp_check_model_file: " + why);
    return DP_ERR_MODEL_FILE;
  }
  return DP_OK;
}

int dp_debug_pair_grads(dp_model *m, int64_t natoms, float *g) {
  if (!m || !g || natoms < 1 || natoms > m->ws.cap) {
    set_error("dp_debug_pair_grads: bad argument");
    return DP_ERR_ARG;
  }
  HIP_TRY(hipSetDevice(m->device));
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(g, m->ws.g, (size_t)natoms * SEL * sizeof(float4), hipMemcpyDeviceToHost));
  return DP_OK;
}

int dp_profile_enable(dp_model *m, int enable) {
  if (!m) return DP_ERR_ARG;
  HIP_TRY(hipSetDevice(m->device));
  if (enable && !m->ev[0])
    for (int k = 0; k < 8; ++k) HIP_TRY(hipEventCreate(&m->ev[k]));
  for (int k = 0; k < 8; ++k) {
    m->prof_ms[k] = 0;
    m->prof_calls[k] = 0;
  }
  m->prof = enable != 0;
  return DP_OK;
}

int dp_profile_read(const dp_model *m, double *ms, int64_t *calls, int max) {
  if (!m) return DP_ERR_ARG;
  for (int k = 0; k < max && k < DP_NPHASES; ++k) {
    if (ms) ms[k] = m->prof_ms[k];
    if (calls) calls[k] = m->prof_calls[k];
  }
  return DP_NPHASES;
}

int dp_model_info(const dp_model *m, double *rc, int *sel, int *ntypes) {
  if (!m) return DP_ERR_ARG;
  if (rc) *rc = m->rc;
  if (sel) *sel = m->sel;
  if (ntypes) *ntypes = m->ntypes;
  return DP_OK;
}

int dp_compute_device(dp_model *m, int64_t natoms, const double *d_coords, const int32_t *d_types,
                      const double *box_host, double *d_energy, double *d_forces, double *d_virial,
                      double *d_atom_energy, void *hip_stream) {
  g_last_error.clear();
  if (!m || natoms < 1 || !d_coords || !d_types || !d_energy) {
    set_error("dp_compute_device: bad argument");
    return DP_ERR_ARG;
  }
  if (natoms > MAX_ATOMS) {
    set_error("natoms above the library limit");
    return DP_ERR_TOO_LARGE;
  }
  HIP_TRY(hipSetDevice(m->device));
  StepArgs a;
  a.n = natoms;
  a.X = d_coords;
  a.types = d_types;
  a.energy = d_energy;
  a.forces = d_forces;
  a.virial = d_virial;
  a.atom_energy = d_atom_energy;
  const int s = run_single(m, a, box_host, (hipStream_t)hip_stream);
  if (s < 0) {
    m->fwd_valid = false;
    return s;
  }
  m->fwd_valid = !(d_forces || d_virial);
  m->fwd_natoms = natoms;
  m->fwd_coords = d_coords;
  m->fwd_types = d_types;
  return s;
}

int dp_compute_owned_device(dp_model *m, int64_t natoms, int64_t n_owned, const double *d_coords,
                            const int32_t *d_types, const double *box_host, double *d_energy, double *d_forces,
                            double *d_virial, double *d_atom_energy, void *hip_stream) {
  g_last_error.clear();
  if (!m || natoms < 1 || n_owned < 0 || n_owned > natoms || !d_coords || !d_types || !d_energy) {
    set_error("dp_compute_owned_device: bad argument");
    return DP_ERR_ARG;
  }
  if (natoms > MAX_ATOMS) {
    set_error("natoms above the library limit");
    return DP_ERR_TOO_LARGE;
  }
  Grid g;
  int s = make_grid(m->rc, m->rc, box_host, g);
  if (s != DP_OK) return s;
  HIP_TRY(hipSetDevice(m->device));
  Workspace &ws = m->ws;
  s = ensure_ws(ws, m->prec, natoms, 1, false);
  if (s != DP_OK) return s;
  ws.grids_host[0] = g;
  ws.off_host[0] = 0;
  ws.off_host[1] = (int)natoms;
  StepArgs a;
  a.n = natoms;
  a.nsys = 1;
  a.n_centres = n_owned;
  a.X = d_coords;
  a.types = d_types;
  a.energy = d_energy;
  a.forces = d_forces;
  a.virial = d_virial;
  a.atom_energy = d_atom_energy;
  a.open_single = box_host == nullptr;
  a.ncells = a.open_single ? MAX_CELLS : g.ncells;
  a.lists = LISTS_FRESH;
  hipStream_t st = (hipStream_t)hip_stream;
  s = enqueue_step(m, ws, a, st, false);
  if (s != DP_OK) return s;
  HIP_TRY(hipMemcpyAsync(ws.flags_host, ws.flags, 4 * sizeof(unsigned), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  m->fwd_valid = false;
  s = step_status(ws);
  // one-sided pairs are expected here (a centre's ghost neighbours have no lists); only a
  // truncated list is a warning
  return s;
}

int dp_compute_device_noalloc(dp_model *m, int64_t natoms, const double *d_coords, const int32_t *d_types,
                              const double *box_host, double *d_energy, double *d_forces, double *d_virial,
                              double *d_atom_energy, void *hip_stream) {
  g_last_error.clear();
  if (!m || natoms < 1 || !d_coords || !d_types || !d_energy) {
    set_error("dp_compute_device_noalloc: bad argument");
    return DP_ERR_ARG;
  }
  if (natoms > DP_NOALLOC_MAX_ATOMS) {
    set_error("dp_compute_device_noalloc: natoms above DP_NOALLOC_MAX_ATOMS (" +
              std::to_string(DP_NOALLOC_MAX_ATOMS) + "); use dp_compute_device");
    return DP_ERR_TOO_LARGE;
  }
  if (m->device < 0 || m->device >= NOALLOC_MAX_DEVICES || !g_noalloc[m->device].ready) {
    set_error("dp_compute_device_noalloc: no allocation-free workspace on this device");
    return DP_ERR_ARG;
  }
  Grid g;
  int s = make_grid(m->rc, m->rc, box_host, g);
  if (s != DP_OK) return s;
  HIP_TRY(hipSetDevice(m->device));
  Workspace &ws = g_noalloc[m->device].ws;
  ws.grids_host[0] = g;
  ws.off_host[0] = 0;
  ws.off_host[1] = (int)natoms;
  StepArgs a;
  a.n = natoms;
  a.nsys = 1;
  a.X = d_coords;
  a.types = d_types;
  a.energy = d_energy;
  a.forces = d_forces;
  a.virial = d_virial;
  a.atom_energy = d_atom_energy;
  a.open_single = box_host == nullptr;
  a.ncells = a.open_single ? MAX_CELLS : g.ncells;
  a.lists = LISTS_FRESH;
  hipStream_t st = (hipStream_t)hip_stream;
  s = enqueue_step(m, ws, a, st, false);
  if (s != DP_OK) return s;
  HIP_TRY(hipMemcpyAsync(ws.flags_host, ws.flags, 4 * sizeof(unsigned), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  m->fwd_valid = false;
  return step_status(ws);
}

int dp_compute_batch_device(dp_model *m, int nsys, const int64_t *natoms, const double *boxes,
                            const double *d_coords, const int32_t *d_types, double *d_energy, double *d_forces,
                            double *d_virial, void *hip_stream) {
  g_last_error.clear();
  if (!m || nsys < 1 || !natoms || !boxes || !d_coords || !d_types || !d_energy) {
    set_error("dp_compute_batch_device: bad argument");
    return DP_ERR_ARG;
  }
  int64_t tot = 0;
  for (int k = 0; k < nsys; ++k) {
    if (natoms[k] < 1) {
      set_error("dp_compute_batch_device: a system has no atoms");
      return DP_ERR_ARG;
    }
    tot += natoms[k];
  }
  if (tot > MAX_ATOMS) {
    set_error("natoms above the library limit");
    return DP_ERR_TOO_LARGE;
  }
  HIP_TRY(hipSetDevice(m->device));
  Workspace &ws = m->ws;
  int s = ensure_ws(ws, m->prec, tot, nsys, false);
  if (s != DP_OK) return s;
  int cells = 0;
  ws.off_host[0] = 0;
  for (int k = 0; k < nsys; ++k) {
    Grid g;
    s = make_grid(m->rc, m->rc, boxes + 9 * k, g);
    if (s != DP_OK) return s;
    if (cells + g.ncells > MAX_CELLS) {
      set_error("dp_compute_batch_device: too many cells in one batch");
      return DP_ERR_TOO_LARGE;
    }
    g.cell_base = cells;
    cells += g.ncells;
    ws.grids_host[k] = g;
    ws.off_host[k + 1] = (int)(ws.off_host[k] + natoms[k]);
  }
  StepArgs a;
  a.n = tot;
  a.nsys = nsys;
  a.X = d_coords;
  a.types = d_types;
  a.energy = d_energy;
  a.forces = d_forces;
  a.virial = d_virial;
  a.ncells = cells;
  a.lists = LISTS_FRESH;
  hipStream_t st = (hipStream_t)hip_stream;
  s = enqueue_step(m, ws, a, st, false);
  if (s != DP_OK) return s;
  HIP_TRY(hipMemcpyAsync(ws.flags_host, ws.flags, 4 * sizeof(unsigned), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  m->fwd_valid = false;
  return step_status(ws);
}

int dp_model_heads(const dp_model *m, int *nheads) {
  if (!m || !nheads) return DP_ERR_ARG;
  *nheads = m->wf.nheads;
  return DP_OK;
}

int dp_set_head_weights(dp_model *m, int nheads, const double *weights) {
  g_last_error.clear();
  if (!m || !weights || nheads != m->wf.nheads) {
    set_error("dp_set_head_weights: bad argument (give one weight per fitting head)");
    return DP_ERR_ARG;
  }
  for (int h = 0; h < nheads; ++h)
    if (!std::isfinite(weights[h])) {
      set_error("dp_set_head_weights: non-finite weight");
      return DP_ERR_NONFINITE;
    }
  HIP_TRY(hipSetDevice(m->device));
  HIP_TRY(hipDeviceSynchronize());
  for (int h = 0; h < nheads; ++h) m->wf.hw[h] = weights[h];
  // the weights travel as kernel arguments: graphs captured with the old ones are dropped
  for (auto &e : m->graphs) {
    if (e.exec) (void)hipGraphExecDestroy(e.exec);
    e.exec = nullptr;
  }
  m->fwd_valid = false;
  return DP_OK;
}

int dp_head_energies(dp_model *m, int nsys, double *energies) {
  g_last_error.clear();
  if (!m || !energies || nsys < 1 || nsys > m->ws.cap_sys || m->wf.nheads < 2) {
    set_error("dp_head_energies: bad argument (a model with several fitting heads and a finished step)");
    return DP_ERR_ARG;
  }
  HIP_TRY(hipSetDevice(m->device));
  HIP_TRY(hipDeviceSynchronize());
  std::vector<double> all((size_t)nsys * MAXH);
  HIP_TRY(hipMemcpy(all.data(), m->ws.Ehsys, all.size() * sizeof(double), hipMemcpyDeviceToHost));
  for (int s = 0; s < nsys; ++s)
    for (int h = 0; h < m->wf.nheads; ++h) energies[s * m->wf.nheads + h] = all[(size_t)s * MAXH + h];
  return DP_OK;
}

int dp_set_skin(dp_model *m, double skin, int rebuild_every) {
  g_last_error.clear();
  if (!m || !(skin >= 0.0) || !std::isfinite(skin) || rebuild_every < 1) {
    set_error("dp_set_skin: bad argument");
    return DP_ERR_ARG;
  }
  m->skin = skin;
  m->rebuild_every = rebuild_every;
  m->skin_valid = false;
  return DP_OK;
}

int dp_skin_stats(const dp_model *m, int64_t *builds, int64_t *forced) {
  if (!m) return DP_ERR_ARG;
  if (builds) *builds = m->skin_builds;
  if (forced) *forced = m->skin_rebuilds_forced;
  return DP_OK;
}

int dp_set_chunk(dp_model *m, int64_t chunk_atoms) {
  g_last_error.clear();
  if (!m || chunk_atoms < 0) {
    set_error("dp_set_chunk: bad argument");
    return DP_ERR_ARG;
  }
  m->chunk = chunk_atoms;
  return DP_OK;
}

int dp_set_graph(dp_model *m, int enable) {
  g_last_error.clear();
  if (!m) return DP_ERR_ARG;
  HIP_TRY(hipSetDevice(m->device));
  HIP_TRY(hipDeviceSynchronize());
  for (auto &e : m->graphs) {
    if (e.exec) (void)hipGraphExecDestroy(e.exec);
    e.exec = nullptr;
  }
  m->use_graph = enable != 0;
  return DP_OK;
}

int dp_backward_device(dp_model *m, const double *d_grad_energy, double *d_grad_coords, double *d_virial,
                       void *hip_stream) {
  g_last_error.clear();
  if (!m || !d_grad_energy || !d_grad_coords) {
    set_error("dp_backward_device: bad argument");
    return DP_ERR_ARG;
  }
  if (!m->fwd_valid) {
    set_error("dp_backward_device: no energy-only forward pass to differentiate");
    return DP_ERR_ARG;
  }
  HIP_TRY(hipSetDevice(m->device));
  hipStream_t st = (hipStream_t)hip_stream;
  const int n = (int)m->fwd_natoms;
  const float rc = (float)m->rc, rcs = (float)m->rcs, eps = (float)m->ln_eps;
  Workspace &ws = m->ws;
  // the energy-only pass left D, the lists and the grid in place; rerun the fitting
  // net with its backward
  if (m->prec == DP_FP32) {
    launch_fitting<float>(m->wf, ws, m->fwd_types, 0, n, true, st);
    launch_descriptor_bwd<float>(m->wf, ws, m->fwd_coords, m->fwd_types, n, 0, n, rc, rcs, eps, st);
  } else {
    launch_fitting_b16(m->wf, m->wp, ws, m->fwd_types, 0, n, true, st);
    launch_descriptor_bwd_b16(m->wf, m->wp, ws, m->fwd_coords, m->fwd_types, n, 0, n, rc, rcs, eps, st);
  }
  launch_forces(ws, m->fwd_coords, n, d_grad_energy, d_grad_coords, m->fwd_lists == LISTS_SKIN_REUSE, false, st);
  if (d_virial) launch_reduce(ws, ws.sys_off, 1, nullptr, nullptr, d_virial, 1, st);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(st));
  m->fwd_valid = false;
  return DP_OK;
}

int dp_compute(dp_model *m, int64_t natoms, const double *coords, const int32_t *types, const double *box,
               double *energy, double *forces, double *virial, double *atom_energy) {
  g_last_error.clear();
  if (!m || natoms < 1 || !coords || !types || !energy) {
    set_error("dp_compute: bad argument");
    return DP_ERR_ARG;
  }
  if (natoms > MAX_ATOMS) {
    set_error("natoms above the library limit");
    return DP_ERR_TOO_LARGE;
  }
  HIP_TRY(hipSetDevice(m->device));
  double *dX = nullptr, *dE = nullptr, *dF = nullptr, *dV = nullptr, *dAE = nullptr;
  int *dT = nullptr;
  const size_t n = (size_t)natoms;
  auto cleanup = [&]() {
    void *ps[] = {dX, dE, dF, dV, dAE, dT};
    for (void *p : ps)
      if (p) (void)hipFree(p);
  };
  if (hipMalloc(&dX, n * 3 * 8) != hipSuccess || hipMalloc(&dT, n * 4) != hipSuccess ||
      hipMalloc(&dE, 8) != hipSuccess || hipMalloc(&dF, n * 3 * 8) != hipSuccess ||
      hipMalloc(&dV, 9 * 8) != hipSuccess || (atom_energy && hipMalloc(&dAE, n * 8) != hipSuccess)) {
    cleanup();
    set_error("dp_compute: device allocation failed");
    return DP_ERR_OOM;
  }
  int s = DP_OK;
  if (hipMemcpy(dX, coords, n * 3 * 8, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(dT, types, n * 4, hipMemcpyHostToDevice) != hipSuccess) {
    cleanup();
    set_error("dp_compute: host to device copy failed");
    return DP_ERR_HIP;
  }
  const bool bwd = forces || virial;
  s = dp_compute_device(m, natoms, dX, dT, box, dE, bwd ? dF : nullptr, bwd ? dV : nullptr, dAE, nullptr);
  if (s >= 0) {
    bool ok = hipMemcpy(energy, dE, 8, hipMemcpyDeviceToHost) == hipSuccess;
    if (forces) ok &= hipMemcpy(forces, dF, n * 3 * 8, hipMemcpyDeviceToHost) == hipSuccess;
    if (virial) ok &= hipMemcpy(virial, dV, 9 * 8, hipMemcpyDeviceToHost) == hipSuccess;
    if (atom_energy) ok &= hipMemcpy(atom_energy, dAE, n * 8, hipMemcpyDeviceToHost) == hipSuccess;
    if (!ok) {
      set_error("dp_compute: device to host copy failed");
      s = DP_ERR_HIP;
    }
  }
  m->fwd_valid = false;
  cleanup();
  return s;
}

int dp_debug_neighbors(dp_model *m, int64_t natoms, const double *coords, const double *box, int32_t *nlist,
                       int32_t *nnei, int64_t *overflow) {
  g_last_error.clear();
  if (!m || natoms < 1 || !coords || !nlist || !nnei) {
    set_error("dp_debug_neighbors: bad argument");
    return DP_ERR_ARG;
  }
  if (natoms > MAX_ATOMS) return DP_ERR_TOO_LARGE;
  Grid g;
  int s = make_grid(m->rc, m->rc, box, g);
  if (s != DP_OK) return s;
  HIP_TRY(hipSetDevice(m->device));
  Workspace &ws = m->ws;
  s = ensure_ws(ws, m->prec, natoms, 1, false);
  if (s != DP_OK) return s;
  const size_t n = (size_t)natoms;
  double *dX = nullptr;
  int *dT = nullptr;
  if (hipMalloc(&dX, n * 24) != hipSuccess || hipMalloc(&dT, n * 4) != hipSuccess) {
    if (dX) (void)hipFree(dX);
    set_error("dp_debug_neighbors: allocation failed");
    return DP_ERR_OOM;
  }
  const bool open = box == nullptr;
  ws.grids_host[0] = g;
  ws.off_host[0] = 0;
  ws.off_host[1] = (int)natoms;
  hipStream_t st = m->own_stream;
  s = DP_OK;
  if (hipMemcpy(dX, coords, n * 24, hipMemcpyHostToDevice) != hipSuccess || hipMemset(dT, 0, n * 4) != hipSuccess ||
      hipMemcpy(ws.grids, ws.grids_host, sizeof(Grid), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(ws.sys_off, ws.off_host, 2 * sizeof(int), hipMemcpyHostToDevice) != hipSuccess) {
    s = DP_ERR_HIP;
  } else {
    launch_prologue(ws, 1, (int)natoms, (open ? MAX_CELLS : g.ncells) + 1, true, st);
    launch_cells(ws, dX, dT, (int)natoms, m->ntypes, open, open ? MAX_CELLS : g.ncells, m->rc, st);
    launch_nlist(ws, dX, (int)natoms, 0, (int)natoms, (int)natoms, m->rc, false, st);
    if (hipStreamSynchronize(st) != hipSuccess ||
        hipMemcpy(nlist, ws.nlist, n * SEL * 4, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(nnei, ws.nnei, n * 4, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(ws.flags_host, ws.flags, 16, hipMemcpyDeviceToHost) != hipSuccess) {
      s = DP_ERR_HIP;
    } else {
      s = flags_status(ws.flags_host[0]);
      if (overflow) *overflow = ws.flags_host[1];
      if (s == DP_OK && ws.flags_host[1]) s = DP_WARN_SEL_OVERFLOW;
    }
  }
  (void)hipFree(dX);
  (void)hipFree(dT);
  m->skin_valid = false;
  if (s == DP_ERR_HIP) set_error("dp_debug_neighbors: HIP call failed");
  return s;
}

}  // extern "C"
