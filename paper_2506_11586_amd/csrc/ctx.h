// Internal: the context object and conv geometry shared by the library's
// host translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "heconv.h"
#include "kernels.h"
#include "modarith.h"

struct he_ctx {
  int device = 0;
  uint32_t N = 0, logN = 0, L = 0;
  uint64_t t = 0;
  bool proto_ok = false;  // t usable by the protocol steps (delta_l != 0)
  std::vector<uint64_t> q, psi;
  std::vector<heconv::LimbConst> lc;
  bool all_pm = false;  // every q_l = 2^60 - delta, delta < 2^20
  heconv::Tw* d_fwd = nullptr;  // [L][N] psi^brv(k) with Shoup quotient
  heconv::Tw* d_inv = nullptr;  // [L][N] psi^-brv(k) with Shoup quotient
  heconv::LimbConst* d_lc = nullptr;
  heconv::DecodeConst* d_dc = nullptr;  // client-side decoding constants (t a power of two)
  // double-precision transforms (every q_l < 2^50)
  bool fp64_ok = false;
  double* d_fwd64 = nullptr;  // [L][N] forward twiddles as doubles
  double* d_inv64 = nullptr;  // [L][N] inverse twiddles as doubles
  void* d_fc = nullptr;       // per-limb F64Const
  bool decode_ok = false;
  heconv::LimbConst tlc{};  // reduction constants of t (decryption)
  he_tuning tune{3, 3, 512, 0, 0, 0, 1, 160, 1, 1, 128, 3, 0, 1};
  // internal stream and events of the output-channel pipeline of he_conv_layer
  hipStream_t aux = nullptr;
  hipEvent_t ev_mac[4] = {nullptr, nullptr, nullptr, nullptr};
  hipEvent_t ev_done = nullptr;
};

namespace heconv {

// Conv geometry derived from a descriptor (mirrors the header's layout).
struct Geo {
  uint32_t He, We, R1, C1, bh, bw, nsi, nsj, S, CB, O;
  bool sub;
};

inline bool geo_of(const he_conv_desc& d, uint32_t N, Geo& g) {
  if (!d.C || !d.H || !d.W || !d.M || !d.kh || !d.kw || !d.stride) return false;
  const uint32_t Hp = d.H + 2 * d.pad, Wp = d.W + 2 * d.pad;
  if (Hp < d.kh || Wp < d.kw) return false;
  const uint32_t Ho = (Hp - d.kh) / d.stride + 1, Wo = (Wp - d.kw) / d.stride + 1;
  g.sub = d.kh == 1 && d.kw == 1 && d.stride > 1;
  if (g.sub) {
    g.He = Ho, g.We = Wo, g.R1 = Ho, g.C1 = Wo;
  } else {
    g.He = Hp, g.We = Wp, g.R1 = (Ho - 1) * d.stride + 1, g.C1 = (Wo - 1) * d.stride + 1;
  }
  if (!d.Cw || !d.Hw || !d.Ww) return false;
  if (d.Cw > d.C || d.Hw < d.kh || d.Ww < d.kw || d.Hw > g.He || d.Ww > g.We) return false;
  if ((uint64_t)d.Cw * d.Hw * d.Ww > N) return false;
  g.bh = d.Hw - d.kh + 1, g.bw = d.Ww - d.kw + 1;
  g.nsi = (g.R1 + g.bh - 1) / g.bh, g.nsj = (g.C1 + g.bw - 1) / g.bw;
  g.S = g.nsi * g.nsj;
  g.CB = (d.C + d.Cw - 1) / d.Cw;
  g.O = (d.Cw - 1) * d.Hw * d.Ww + (d.kh - 1) * d.Ww + (d.kw - 1);
  return true;
}

// The MAC addresses one image's input ciphertexts and one output channel's
// weights with 32-bit byte offsets below 2^31.
inline bool mac_offsets_fit(const Geo& g, uint32_t L, uint32_t N) {
  const uint64_t LN8 = (uint64_t)L * N * 8;
  return (uint64_t)g.CB * g.S * 2 * LN8 < (1ull << 31) && (uint64_t)g.CB * LN8 < (1ull << 31);
}

}  // namespace heconv
