// C ABI of the homomorphic-convolution library (declared in include/heconv.h):
// parameter checks, the library's own prime/root search and twiddle tables,
// the packing planner, and the entry points that enqueue the HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "heconv.h"
#include "ctx.h"
#include "kernels.h"

using heconv::LimbConst;
using heconv::Tw;
using heconv::Geo;
using heconv::geo_of;

namespace {

typedef unsigned __int128 u128;

uint64_t mmul(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((u128)a * b % m); }

uint64_t mpow(uint64_t b, uint64_t e, uint64_t m) {
  uint64_t r = 1;
  b %= m;
  for (; e; e >>= 1, b = mmul(b, b, m))
    if (e & 1) r = mmul(r, b, m);
  return r;
}

// Miller-Rabin with the seven bases of Jaeschke/Sinclair, exact for all
// 64-bit inputs.
bool prime64(uint64_t n) {
  if (n < 2) return false;
  for (uint64_t p : {2ull, 3ull, 5ull, 7ull, 11ull, 13ull, 17ull, 19ull, 23ull, 29ull, 31ull, 37ull}) {
    if (n % p == 0) return n == p;
  }
  uint64_t d = n - 1;
  unsigned s = __builtin_ctzll(d);
  d >>= s;
  for (uint64_t a : {2ull, 325ull, 9375ull, 28178ull, 450775ull, 9780504ull, 1795265022ull}) {
    uint64_t x = mpow(a % n, d, n);
    if (x == 0 || x == 1 || x == n - 1) continue;
    bool comp = true;
    for (unsigned r = 1; r < s && comp; r++) {
      x = mmul(x, x, n);
      if (x == n - 1) comp = false;
    }
    if (comp) return false;
  }
  return true;
}

bool pow2(uint64_t x) { return x && !(x & (x - 1)); }

unsigned log2u(uint64_t x) { return 63 - __builtin_clzll(x); }

unsigned bitrev(unsigned x, unsigned bits) {
  unsigned r = 0;
  for (unsigned i = 0; i < bits; i++, x >>= 1) r = (r << 1) | (x & 1);
  return r;
}

// The smallest primitive 2N-th root of unity mod q (q = 1 mod 2N).  A
// primitive 2N-th root r is c^((q-1)/2N) for some c with r^N = -1; every
// other is an odd power of r.
uint64_t min_root(uint64_t q, uint32_t N) {
  uint64_t r = 0;
  for (uint64_t c = 2; c < q && !r; c++) {
    uint64_t cand = mpow(c, (q - 1) / (2ull * N), q);
    if (mpow(cand, N, q) == q - 1) r = cand;
  }
  if (!r) return 0;
  const uint64_t r2 = mmul(r, r, q);
  uint64_t best = r;
  for (uint64_t k = 1, v = r; k < 2ull * N; k += 2, v = mmul(v, r2, q))
    if (v < best) best = v;
  return best;
}

uint64_t shoup(uint64_t w, uint64_t q) { return (uint64_t)(((u128)w << 64) / q); }

// Shoup quotient at scale 2^63 (the transforms' twiddle tables).
uint64_t shoup63(uint64_t w, uint64_t q) { return (uint64_t)(((u128)w << 63) / q); }

// delta_l = floor(Q/t) mod q_l for Q = prod q_l, in multi-word arithmetic
// (little-endian 64-bit words).  All zero when t is outside [2, 2^62] or
// t > Q: the protocol steps then refuse to run.
std::vector<uint64_t> deltas(const std::vector<uint64_t>& q, uint64_t t) {
  std::vector<uint64_t> out(q.size(), 0);
  if (t < 2 || t > (1ull << 62)) return out;
  std::vector<uint64_t> Q{1};
  for (uint64_t ql : q) {
    u128 carry = 0;
    for (uint64_t& w : Q) {
      const u128 p = (u128)w * ql + carry;
      w = (uint64_t)p;
      carry = p >> 64;
    }
    if (carry) Q.push_back((uint64_t)carry);
  }
  std::vector<uint64_t> D(Q.size());
  u128 rem = 0;
  bool nonzero = false;
  for (size_t i = Q.size(); i-- > 0;) {
    const u128 cur = (rem << 64) | Q[i];
    D[i] = (uint64_t)(cur / t);
    rem = cur % t;
    nonzero |= D[i] != 0;
  }
  if (!nonzero) return out;
  for (size_t l = 0; l < q.size(); l++) {
    u128 r = 0;
    for (size_t i = D.size(); i-- > 0;) r = ((r << 64) | D[i]) % q[l];
    out[l] = (uint64_t)r;
  }
  return out;
}

}  // namespace

namespace {

he_status check_ctx(const he_ctx* c) { return c ? HE_OK : HE_EINVAL; }

uint32_t ntt_loge(const he_ctx* c, uint64_t n_rns_polys) {
  return n_rns_polys * c->L < c->tune.ntt_small_below ? c->tune.ntt_loge_small : c->tune.ntt_loge_large;
}

he_status dev_err(hipError_t e) { return e == hipSuccess ? HE_OK : HE_EDEVICE; }

// Every transform of the library goes through here: double precision when
// all primes allow it (and the tuning asks for it), else the integer
// kernels -- for a small count, in two grids.
hipError_t ntt_run(const he_ctx* c, bool inverse, uint64_t* polys, uint64_t n, hipStream_t st, bool nt = false) {
  if (c->fp64_ok && c->tune.ntt_fp64)
    return heconv::ntt_f64_launch(inverse, c->logN, ntt_loge(c, n), polys, n, c->L, inverse ? c->d_inv64 : c->d_fwd64,
                                  c->d_fc, st);
  if (!inverse && n * c->L < c->tune.ntt_split_below && heconv::ntt_fwd_split_supported(c->logN))
    return heconv::ntt_fwd_split_launch(c->logN, polys, n, c->L, c->d_fwd, c->d_lc, st);
  if (inverse && n * c->L < c->tune.ntt_inv_split_below && heconv::ntt_inv_split_supported(c->logN))
    return heconv::ntt_inv_split_launch(c->logN, polys, n, c->L, c->d_inv, c->d_lc, st);
  return heconv::ntt_launch(inverse, c->logN, ntt_loge(c, n), polys, n, c->L, inverse ? c->d_inv : c->d_fwd, c->d_lc,
                            st, nt);
}

}  // namespace

extern "C" {

const char* he_status_str(he_status s) {
  switch (s) {
    case HE_OK: return "ok";
    case HE_EINVAL: return "invalid argument";
    case HE_ESHAPE: return "shape/descriptor mismatch";
    case HE_EPARAM: return "unsupported parameters";
    case HE_ENOMEM: return "device allocation failed";
    case HE_EDEVICE: return "HIP device error";
    case HE_EBUSY: return "busy";
  }
  return "unknown status";
}

he_status he_gen_primes(uint32_t N, uint32_t bits, uint32_t L, uint64_t* q_out) {
  if (!q_out || !pow2(N) || N < 2 || bits < 20 || bits > 60 || L == 0) return HE_EPARAM;
  const uint64_t m = 2ull * N;
  uint64_t c = ((1ull << bits) - 2) / m * m + 1;  // largest value below 2^bits that is 1 mod 2N
  uint32_t got = 0;
  for (; got < L && c > m; c -= m)
    if (prime64(c)) q_out[got++] = c;
  return got == L ? HE_OK : HE_EPARAM;
}

he_status he_ctx_create(const he_params* prm, he_ctx** out) {
  if (!prm || !out || !prm->q) return HE_EINVAL;
  *out = nullptr;
  const uint32_t N = prm->N, L = prm->L;
  if (!pow2(N) || N < (1u << 10) || N > (1u << 14) || L == 0 || L > 8) return HE_EPARAM;
  for (uint32_t l = 0; l < L; l++) {
    const uint64_t q = prm->q[l];
    if (q >= (1ull << 60) || q % (2ull * N) != 1 || !prime64(q)) return HE_EPARAM;
    for (uint32_t j = 0; j < l; j++)
      if (prm->q[j] == q) return HE_EPARAM;
  }
  he_ctx* c = new (std::nothrow) he_ctx;
  if (!c) return HE_ENOMEM;
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return HE_EDEVICE;
  }
  c->N = N, c->logN = log2u(N), c->L = L, c->t = prm->t;
  c->q.assign(prm->q, prm->q + L);
  const std::vector<uint64_t> dl = deltas(c->q, c->t);
  c->proto_ok = std::all_of(dl.begin(), dl.end(), [](uint64_t v) { return v != 0; });
  std::vector<Tw> fwd((size_t)L * N), inv((size_t)L * N);
  std::vector<uint64_t> pw(N);
  for (uint32_t l = 0; l < L; l++) {
    const uint64_t q = c->q[l];
    const uint64_t psi = min_root(q, N);
    if (!psi) {
      delete c;
      return HE_EPARAM;
    }
    c->psi.push_back(psi);
    const uint64_t psi_inv = mpow(psi, q - 2, q);
    for (int dir = 0; dir < 2; dir++) {
      const uint64_t base = dir ? psi_inv : psi;
      pw[0] = 1;
      for (uint32_t i = 1; i < N; i++) pw[i] = mmul(pw[i - 1], base, q);
      Tw* tab = (dir ? inv.data() : fwd.data()) + (size_t)l * N;
      for (uint32_t k = 0; k < N; k++) {
        const uint64_t w = pw[bitrev(k, c->logN)];
        tab[k] = Tw{w, shoup63(w, q)};
      }
    }
    LimbConst k{};
    k.q = q, k.two_q = 2 * q;
    k.ninv = mpow(N % q, q - 2, q), k.ninv_sh = shoup(k.ninv, q);
    k.ninv_w = mmul(k.ninv, inv[(size_t)l * N + 1].w, q), k.ninv_w_sh = shoup(k.ninv_w, q);
    k.r64 = (uint64_t)(((u128)1 << 64) % q), k.r64_sh = shoup(k.r64, q), k.r64_sh63 = shoup63(k.r64, q);
    k.mu64 = (uint64_t)(((u128)1 << 64) / q);
    k.c30 = (uint64_t)(((u128)1 << 30) % q), k.c30_sh = shoup(k.c30, q);
    k.c60 = (uint64_t)(((u128)1 << 60) % q), k.c60_sh = shoup(k.c60, q);
    k.delta = dl[l], k.delta_sh = shoup(dl[l], q);
    k.negq = 0 - q, k.neg2q = 0 - 2 * q;
    k.three_q = 3 * q, k.neg3q = 0 - 3 * q;
    // the MAC's folds for q = 2^60 - delta, delta < 2^20 (modarith.h, fold30_pm, fold3_pm)
    k.pmd = (q < (1ull << 60) && (1ull << 60) - q < (1ull << 20)) ? (1ull << 60) - q : 0;
    c->lc.push_back(k);
  }
  c->all_pm = true;
  for (const heconv::LimbConst& k : c->lc) c->all_pm &= k.pmd != 0;
  // client-side decoding constants (power-of-two t only)
  std::vector<heconv::DecodeConst> dc(L);
  c->decode_ok = c->proto_ok && c->t >= 2 && c->t < (1ull << 62);
  if (c->decode_ok) {
    const uint64_t t = c->t;
    c->tlc.q = t, c->tlc.two_q = 2 * t;
    c->tlc.r64 = (uint64_t)(((u128)1 << 64) % t), c->tlc.r64_sh = shoup(c->tlc.r64, t);
    c->tlc.mu64 = (uint64_t)(((u128)1 << 64) / t);
  }
  for (uint32_t l = 0; l < L && c->decode_ok; l++) {
    const uint64_t q = c->q[l];
    uint64_t qh = 1;
    for (uint32_t j = 0; j < L; j++)
      if (j != l) qh = mmul(qh, c->q[j] % q, q);
    const uint64_t y = mpow(qh, q - 2, q);
    const u128 ty = (u128)c->t * y;
    const uint64_t r = (uint64_t)(ty % q);
    const u128 r64 = (u128)r << 64;
    const uint64_t fh = (uint64_t)(r64 / q), r2 = (uint64_t)(r64 % q);
    dc[l] = heconv::DecodeConst{(uint64_t)(ty / q), fh, (uint64_t)(((u128)r2 << 64) / q)};
  }
  // double-precision transforms when every prime is below 2^50
  c->fp64_ok = std::all_of(c->q.begin(), c->q.end(), [](uint64_t q) { return q < (1ull << 50); });
  std::vector<double> fwd64, inv64;
  std::vector<unsigned char> fc;
  if (c->fp64_ok) {
    fwd64.resize((size_t)L * N), inv64.resize((size_t)L * N), fc.resize(heconv::f64_const_size() * L);
    for (size_t i = 0; i < (size_t)L * N; i++) fwd64[i] = (double)fwd[i].w, inv64[i] = (double)inv[i].w;
    for (uint32_t l = 0; l < L; l++)
      heconv::f64_const_fill(fc.data() + heconv::f64_const_size() * l, (double)c->q[l], 1.0 / (double)c->q[l],
                             (double)c->lc[l].ninv, (double)c->lc[l].ninv_w);
  }
  const size_t tb = sizeof(Tw) * (size_t)L * N;
  if (hipMalloc(&c->d_fwd, tb) != hipSuccess || hipMalloc(&c->d_inv, tb) != hipSuccess ||
      hipMalloc(&c->d_lc, sizeof(LimbConst) * L) != hipSuccess ||
      hipMalloc(&c->d_dc, sizeof(heconv::DecodeConst) * L) != hipSuccess ||
      (c->fp64_ok && (hipMalloc(&c->d_fwd64, sizeof(double) * L * N) != hipSuccess ||
                      hipMalloc(&c->d_inv64, sizeof(double) * L * N) != hipSuccess ||
                      hipMalloc(&c->d_fc, fc.size()) != hipSuccess))) {
    he_ctx_destroy(c);
    return HE_ENOMEM;
  }
  bool ok_ev = hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking) == hipSuccess &&
               hipEventCreateWithFlags(&c->ev_done, hipEventDisableTiming) == hipSuccess;
  for (int i = 0; i < 4 && ok_ev; i++)
    ok_ev = hipEventCreateWithFlags(&c->ev_mac[i], hipEventDisableTiming) == hipSuccess;
  if (!ok_ev) {
    he_ctx_destroy(c);
    return HE_EDEVICE;
  }
  if (hipMemcpy(c->d_fwd, fwd.data(), tb, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->d_inv, inv.data(), tb, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->d_lc, c->lc.data(), sizeof(LimbConst) * L, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->d_dc, dc.data(), sizeof(heconv::DecodeConst) * L, hipMemcpyHostToDevice) != hipSuccess ||
      (c->fp64_ok &&
       (hipMemcpy(c->d_fwd64, fwd64.data(), sizeof(double) * L * N, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->d_inv64, inv64.data(), sizeof(double) * L * N, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->d_fc, fc.data(), fc.size(), hipMemcpyHostToDevice) != hipSuccess))) {
    he_ctx_destroy(c);
    return HE_EDEVICE;
  }
  *out = c;
  return HE_OK;
}

void he_ctx_destroy(he_ctx* c) {
  if (!c) return;
  if (c->d_fwd) (void)hipFree(c->d_fwd);
  if (c->d_inv) (void)hipFree(c->d_inv);
  if (c->d_lc) (void)hipFree(c->d_lc);
  if (c->d_dc) (void)hipFree(c->d_dc);
  if (c->d_fwd64) (void)hipFree(c->d_fwd64);
  if (c->d_inv64) (void)hipFree(c->d_inv64);
  if (c->d_fc) (void)hipFree(c->d_fc);
  for (int i = 0; i < 4; i++)
    if (c->ev_mac[i]) (void)hipEventDestroy(c->ev_mac[i]);
  if (c->ev_done) (void)hipEventDestroy(c->ev_done);
  if (c->aux) (void)hipStreamDestroy(c->aux);
  delete c;
}

he_status he_ctx_psi(const he_ctx* c, uint64_t* psi_out) {
  if (check_ctx(c) || !psi_out) return HE_EINVAL;
  std::memcpy(psi_out, c->psi.data(), sizeof(uint64_t) * c->L);
  return HE_OK;
}

he_status he_ctx_get_tuning(const he_ctx* c, he_tuning* out) {
  if (check_ctx(c) || !out) return HE_EINVAL;
  *out = c->tune;
  return HE_OK;
}

he_status he_ctx_set_tuning(he_ctx* c, const he_tuning* t) {
  if (check_ctx(c) || !t) return HE_EINVAL;
  auto loge_ok = [](uint32_t v) { return v == 3 || v == 4; };
  if (!loge_ok(t->ntt_loge_small) || !loge_ok(t->ntt_loge_large)) return HE_EINVAL;
  static const uint32_t tiles[][2] = {{0, 0}, {4, 4}, {4, 2}, {2, 4}, {8, 2}, {2, 8}, {8, 1}, {1, 8}, {2, 2},
                                      {6, 4}, {8, 4}, {4, 8}};
  bool ok = false;
  for (auto& p : tiles) ok |= (p[0] == t->mac_mt && p[1] == t->mac_rt);
  if (!ok || t->layer_fused > 1 || t->ntt_fp64 > 1 || t->ks_fused > 2) return HE_EINVAL;
  if (t->layer_split != 1 && t->layer_split != 2 && t->layer_split != 4) return HE_EINVAL;
  if (t->mac_lds == 1 || t->mac_lds > 4 || t->mac_tiles > 64 || t->mac_grid > 1) return HE_EINVAL;
  c->tune = *t;
  return HE_OK;
}

namespace {

// The planner's objective for a planned layer: HBM bytes (weights once,
// inputs and outputs three times each per image) and modmuls.
void plan_cost(const he_conv_desc& d, const Geo& g, uint32_t N, uint32_t L, uint32_t B, u128& bytes, u128& mm) {
  const u128 LN8 = (u128)L * N * 8, ct = 2 * LN8;
  const u128 ntt_mm = (u128)L * (N / 2) * log2u(N) * 2;  // per ciphertext
  const u128 in_cts = (u128)g.CB * g.S, out_cts = (u128)d.M * g.S;
  bytes = (u128)d.M * g.CB * LN8 + (u128)B * 3 * (in_cts + out_cts) * ct;
  mm = (u128)B * (in_cts + out_cts) * ntt_mm + (u128)B * d.M * g.CB * g.S * 2 * L * N;
}

}  // namespace

he_status he_plan_conv_host(uint32_t N, uint32_t L, he_conv_desc* io, uint32_t batch_hint) {
  if (!io) return HE_EINVAL;
  if (!pow2(N) || N < 2 || L == 0) return HE_EPARAM;
  if (!batch_hint) batch_hint = 1;
  he_conv_desc d = *io;
  d.Cw = 1, d.Hw = d.kh, d.Ww = d.kw;
  Geo g0;
  if (!geo_of(d, N, g0)) return io->C && io->M && io->kh && io->kw && io->stride ? HE_ESHAPE : HE_EINVAL;
  bool have = false;
  u128 best_b = 0, best_m = 0;
  uint32_t bHw = 0, bWw = 0, bCw = 0;
  for (uint32_t Hw = d.kh; Hw <= g0.He; Hw++) {
    for (uint32_t Ww = d.kw; Ww <= g0.We; Ww++) {
      if ((uint64_t)Hw * Ww > N) break;
      d.Hw = Hw, d.Ww = Ww;
      d.Cw = std::min<uint64_t>(d.C, N / ((uint64_t)Hw * Ww));
      Geo g;
      if (!geo_of(d, N, g)) continue;
      u128 bytes, mm;
      plan_cost(d, g, N, L, batch_hint, bytes, mm);
      // strict improvement keeps the earlier (smaller) Hw/Ww on ties of both
      // costs; ties are then broken towards larger Hw, then larger Ww
      bool better = !have || bytes < best_b || (bytes == best_b && mm < best_m) ||
                    (bytes == best_b && mm == best_m && (Hw > bHw || (Hw == bHw && Ww > bWw)));
      if (better) have = true, best_b = bytes, best_m = mm, bHw = Hw, bWw = Ww, bCw = d.Cw;
    }
  }
  if (!have) return HE_ESHAPE;
  io->Cw = bCw, io->Hw = bHw, io->Ww = bWw;
  return HE_OK;
}

he_status he_plan_conv(const he_ctx* c, he_conv_desc* io, uint32_t batch_hint) {
  if (check_ctx(c)) return HE_EINVAL;
  return he_plan_conv_host(c->N, c->L, io, batch_hint);
}

he_status he_min_root(uint64_t q, uint32_t N, uint64_t* psi_out) {
  if (!psi_out || !pow2(N) || N < 2 || q % (2ull * N) != 1 || q >= (1ull << 62) || !prime64(q)) return HE_EPARAM;
  *psi_out = min_root(q, N);
  return *psi_out ? HE_OK : HE_EPARAM;
}

he_status he_conv_sizes(const he_ctx* c, const he_conv_desc* d, uint32_t* CB, uint32_t* S, uint64_t* in_cts,
                        uint64_t* out_cts, uint64_t* w_words) {
  if (check_ctx(c) || !d) return HE_EINVAL;
  Geo g;
  if (!geo_of(*d, c->N, g)) return HE_ESHAPE;
  if (CB) *CB = g.CB;
  if (S) *S = g.S;
  if (in_cts) *in_cts = (uint64_t)g.CB * g.S;
  if (out_cts) *out_cts = (uint64_t)d->M * g.S;
  if (w_words) *w_words = (uint64_t)d->M * g.CB * c->L * c->N;
  return HE_OK;
}

he_status he_encode_weights(const he_ctx* c, const he_conv_desc* d, const int64_t* d_w, uint64_t* d_wntt,
                            void* stream) {
  if (check_ctx(c) || !d || !d_w || !d_wntt) return HE_EINVAL;
  Geo g;
  if (!geo_of(*d, c->N, g)) return HE_ESHAPE;
  heconv::PackGeom pg{d->M, d->C, d->kh, d->kw, d->Cw, d->Hw, d->Ww, g.CB, c->L, c->N, g.O};
  hipStream_t st = (hipStream_t)stream;
  he_status s = dev_err(heconv::pack_weights_launch(pg, d_w, d_wntt, c->d_lc, st));
  if (s) return s;
  return dev_err(ntt_run(c, false, d_wntt, (uint64_t)d->M * g.CB, st));
}

he_status he_ntt_fwd(const he_ctx* c, uint64_t* d_polys, uint64_t n, void* stream) {
  if (check_ctx(c)) return HE_EINVAL;
  if (n == 0) return HE_OK;
  if (!d_polys) return HE_EINVAL;
  return dev_err(ntt_run(c, false, d_polys, n, (hipStream_t)stream));
}

he_status he_ntt_inv(const he_ctx* c, uint64_t* d_polys, uint64_t n, void* stream) {
  if (check_ctx(c)) return HE_EINVAL;
  if (n == 0) return HE_OK;
  if (!d_polys) return HE_EINVAL;
  return dev_err(ntt_run(c, true, d_polys, n, (hipStream_t)stream, true));
}

he_status he_conv_ntt_mac(const he_ctx* c, const he_conv_desc* d, uint32_t B, const uint64_t* d_in_ntt,
                          const uint64_t* d_wntt, uint64_t* d_out_ntt, void* stream) {
  if (check_ctx(c) || !d) return HE_EINVAL;
  Geo g;
  if (!geo_of(*d, c->N, g)) return HE_ESHAPE;
  if (B == 0) return HE_OK;
  if (!d_in_ntt || !d_wntt || !d_out_ntt) return HE_EINVAL;
  if ((uint64_t)B * g.S * 2 > 0xffffffffull || !heconv::mac_offsets_fit(g, c->L, c->N)) return HE_ESHAPE;
  return dev_err(heconv::mac_launch(d_in_ntt, d_wntt, d_out_ntt, B, g.CB, g.S, d->M, c->L, c->N, c->d_lc,
                                    c->tune.mac_mt, c->tune.mac_rt, c->tune.mac_lds, c->all_pm, c->tune.mac_grid != 0,
                                    (hipStream_t)stream));
}

he_status he_conv_mac_intt(const he_ctx* c, const he_conv_desc* d, uint32_t B, const uint64_t* d_in_ntt,
                           const uint64_t* d_wntt, uint64_t* d_out, void* stream) {
  if (check_ctx(c) || !d) return HE_EINVAL;
  Geo g;
  if (!geo_of(*d, c->N, g)) return HE_ESHAPE;
  if (B == 0) return HE_OK;
  if (!d_in_ntt || !d_wntt || !d_out) return HE_EINVAL;
  return dev_err(heconv::mac_intt_launch(c->logN, d_in_ntt, d_wntt, d_out, B, g.CB, g.S, d->M, c->L, c->d_inv,
                                         c->d_lc, (hipStream_t)stream));
}

he_status he_conv_layer(const he_ctx* c, const he_conv_desc* d, uint32_t B, uint64_t* d_in, const uint64_t* d_wntt,
                        uint64_t* d_out, void* stream) {
  if (check_ctx(c) || !d) return HE_EINVAL;
  Geo g;
  if (!geo_of(*d, c->N, g)) return HE_ESHAPE;
  if (B == 0) return HE_OK;
  if (!d_in || !d_wntt || !d_out) return HE_EINVAL;
  if ((uint64_t)B * g.S * 2 > 0xffffffffull || !heconv::mac_offsets_fit(g, c->L, c->N)) return HE_ESHAPE;
  hipStream_t st = (hipStream_t)stream;
  he_status s = he_ntt_fwd(c, d_in, (uint64_t)B * g.CB * g.S * 2, stream);
  if (s) return s;
  if (c->tune.layer_fused) return he_conv_mac_intt(c, d, B, d_in, d_wntt, d_out, stream);
  const uint32_t P = c->tune.layer_split;
  if (P == 1 || B != 1 || d->M < 8 * P) {
    s = he_conv_ntt_mac(c, d, B, d_in, d_wntt, d_out, stream);
    if (s) return s;
    return he_ntt_inv(c, d_out, (uint64_t)B * d->M * g.S * 2, stream);
  }
  // One image: output channels in slices (contiguous in the weights and in
  // the output).  The slices' MACs run one after another on the caller's
  // stream; the inverse NTT of slice p runs on the context's internal
  // stream once MAC p is done, beside MAC p+1 (HBM-bound MAC, VALU-bound
  // transform).  The caller's stream then waits for the last transform.
  const uint64_t w_per_m = (uint64_t)g.CB * c->L * c->N, out_per_m = (uint64_t)g.S * 2 * c->L * c->N;
  uint32_t m0 = 0;
  for (uint32_t p = 0; p < P; p++) {
    // slice boundaries on multiples of 4 (the MAC's channel tile)
    const uint32_t m_end = p + 1 == P ? d->M : (uint32_t)((uint64_t)d->M * (p + 1) / P) & ~3u;
    const uint32_t Mp = m_end - m0;
    s = dev_err(heconv::mac_launch(d_in, d_wntt + m0 * w_per_m, d_out + m0 * out_per_m, 1, g.CB, g.S, Mp, c->L,
                                   c->N, c->d_lc, c->tune.mac_mt, c->tune.mac_rt, c->tune.mac_lds, c->all_pm,
                                   c->tune.mac_grid != 0, st));
    if (s) return s;
    if (hipEventRecord(c->ev_mac[p], st) != hipSuccess || hipStreamWaitEvent(c->aux, c->ev_mac[p], 0) != hipSuccess)
      return HE_EDEVICE;
    s = dev_err(ntt_run(c, true, d_out + m0 * out_per_m, (uint64_t)Mp * g.S * 2, c->aux, true));
    if (s) return s;
    m0 = m_end;
  }
  if (hipEventRecord(c->ev_done, c->aux) != hipSuccess || hipStreamWaitEvent(st, c->ev_done, 0) != hipSuccess)
    return HE_EDEVICE;
  return HE_OK;
}

namespace {

// Geometry of the protocol kernels; HE_ESHAPE for an invalid descriptor.
he_status proto_geom(const he_ctx* c, const he_conv_desc* d, uint32_t B, heconv::ProtoGeom& p) {
  Geo g;
  if (!geo_of(*d, c->N, g) || d->pad > (1u << 20) || d->H > (1u << 20) || d->W > (1u << 20)) return HE_ESHAPE;
  p = heconv::ProtoGeom{};
  p.B = B, p.C = d->C, p.H = d->H, p.W = d->W, p.M = d->M, p.Cw = d->Cw, p.Hw = d->Hw, p.Ww = d->Ww;
  p.bh = g.bh, p.bw = g.bw, p.nsj = g.nsj, p.S = g.S, p.CB = g.CB, p.O = g.O, p.He = g.He, p.We = g.We;
  p.Ho = (d->H + 2 * d->pad - d->kh) / d->stride + 1, p.Wo = (d->W + 2 * d->pad - d->kw) / d->stride + 1;
  p.step = g.sub ? d->stride : 1, p.ostep = g.sub ? 1 : d->stride;
  p.pad = (int32_t)d->pad, p.L = c->L, p.N = c->N, p.t = c->t;
  return HE_OK;
}

}  // namespace

he_status he_delta_host(const uint64_t* q, uint32_t L, uint64_t t, uint64_t* delta_out) {
  if (!q || !delta_out || L == 0 || L > 8) return HE_EINVAL;
  const std::vector<uint64_t> dl = deltas(std::vector<uint64_t>(q, q + L), t);
  if (!std::all_of(dl.begin(), dl.end(), [](uint64_t v) { return v != 0; })) return HE_EPARAM;
  std::copy(dl.begin(), dl.end(), delta_out);
  return HE_OK;
}

he_status he_add_share(const he_ctx* c, const he_conv_desc* d, uint32_t B, uint64_t* d_in, const int64_t* d_share,
                       void* stream) {
  if (check_ctx(c) || !d) return HE_EINVAL;
  heconv::ProtoGeom p;
  if (he_status s = proto_geom(c, d, B, p)) return s;
  if (!c->proto_ok) return HE_EPARAM;
  if (B == 0) return HE_OK;
  if (!d_in || !d_share) return HE_EINVAL;
  return dev_err(heconv::add_share_launch(d_in, d_share, p, c->d_lc, (hipStream_t)stream));
}

he_status he_mask_extract(const he_ctx* c, const he_conv_desc* d, uint32_t B, const uint64_t* d_out,
                          const int64_t* d_mask, const int64_t* d_noise, uint64_t* d_y, void* stream) {
  if (check_ctx(c) || !d) return HE_EINVAL;
  heconv::ProtoGeom p;
  if (he_status s = proto_geom(c, d, B, p)) return s;
  if (!c->proto_ok) return HE_EPARAM;
  if (B == 0) return HE_OK;
  if (!d_out || !d_mask || !d_y) return HE_EINVAL;
  return dev_err(heconv::mask_extract_launch(d_out, d_mask, d_noise, d_y, p, c->d_lc, (hipStream_t)stream));
}

// ---- client side (secret key on the device) ----

he_status he_key_encode(const he_ctx* c, const int64_t* d_sk, uint64_t* d_sk_ntt, void* stream) {
  if (check_ctx(c) || !d_sk || !d_sk_ntt) return HE_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  he_status s = dev_err(heconv::key_lift_launch(d_sk, d_sk_ntt, c->N, c->L, c->d_lc, st));
  if (s) return s;
  return dev_err(ntt_run(c, false, d_sk_ntt, 1, st));
}

namespace {

// work[i] = a * sk (coefficient form) for the a polynomials at src (stride
// src_stride words); with ct_out, a is also copied to ct_out[i][0].
he_status key_product(const he_ctx* c, uint64_t n, const uint64_t* src, uint64_t src_stride, uint64_t* ct_out,
                      const uint64_t* sk_ntt, uint64_t* work, hipStream_t st) {
  he_status s = dev_err(heconv::copy_a_launch(src, src_stride, work, ct_out, n, c->N, c->L, st));
  if (!s) s = dev_err(ntt_run(c, false, work, n, st));
  if (!s) s = dev_err(heconv::pointwise_key_launch(work, sk_ntt, n, c->N, c->L, c->d_lc, st));
  if (!s) s = dev_err(ntt_run(c, true, work, n, st));
  return s;
}

constexpr uint64_t CLIENT_CHUNK = 65535;  // RNS polynomials per launch (grid.y)

}  // namespace

he_status he_encrypt(const he_ctx* c, uint64_t n, const int64_t* d_msgs, const uint64_t* d_a, const int64_t* d_err,
                     const uint64_t* d_sk_ntt, uint64_t* d_ct, uint64_t* d_work, void* stream) {
  if (check_ctx(c)) return HE_EINVAL;
  if (!c->proto_ok) return HE_EPARAM;
  if (n == 0) return HE_OK;
  if (!d_msgs || !d_a || !d_err || !d_sk_ntt || !d_ct || !d_work) return HE_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const uint64_t LN = (uint64_t)c->L * c->N;
  for (uint64_t i0 = 0; i0 < n; i0 += CLIENT_CHUNK) {
    const uint64_t m = n - i0 < CLIENT_CHUNK ? n - i0 : CLIENT_CHUNK;
    uint64_t* ct = d_ct + i0 * 2 * LN;
    he_status s = key_product(c, m, d_a + i0 * LN, LN, ct, d_sk_ntt, d_work, st);
    if (!s)
      s = dev_err(heconv::encrypt_finish_launch(d_work, d_msgs + i0 * c->N, d_err + i0 * c->N, ct, m, c->N, c->L,
                                                c->t, c->d_lc, st));
    if (s) return s;
  }
  return HE_OK;
}

he_status he_decrypt(const he_ctx* c, uint64_t n, const uint64_t* d_ct, const uint64_t* d_sk_ntt, int64_t* d_msgs,
                     uint64_t* d_work, void* stream) {
  if (check_ctx(c)) return HE_EINVAL;
  if (!c->decode_ok) return HE_EPARAM;
  if (n == 0) return HE_OK;
  if (!d_ct || !d_sk_ntt || !d_msgs || !d_work) return HE_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const uint64_t LN = (uint64_t)c->L * c->N;
  for (uint64_t i0 = 0; i0 < n; i0 += CLIENT_CHUNK) {
    const uint64_t m = n - i0 < CLIENT_CHUNK ? n - i0 : CLIENT_CHUNK;
    const uint64_t* ct = d_ct + i0 * 2 * LN;
    he_status s = key_product(c, m, ct, 2 * LN, nullptr, d_sk_ntt, d_work, st);
    if (!s)
      s = dev_err(heconv::decrypt_finish_launch(ct, d_work, d_msgs + i0 * c->N, m, c->N, c->L, c->tlc, c->d_dc,
                                                c->d_lc, st));
    if (s) return s;
  }
  return HE_OK;
}

// ---- rotation for the Z_P variant (extended context: q_0..q_{L-1}, P) ----

namespace {

// largest grid of the rotation kernels (workgroups of up to N/8 = 1024 threads)
constexpr uint64_t ROT_MAX_BLOCKS = heconv::grid_max_blocks(1024);

// g^-1 mod 2N for odd g (the odd residues mod 2N form a group).
uint32_t inv_mod_2n(uint64_t g, uint32_t N) {
  const uint64_t m = 2ull * N;
  uint64_t r = 1;
  for (uint64_t e = m / 2 - 1, b = g % m; e; e >>= 1, b = b * b % m)
    if (e & 1) r = r * b % m;
  return (uint32_t)r;
}

bool galois_ok(uint64_t g, uint32_t N) { return (g & 1) && g < 2ull * N; }

// Shape checks shared by key switching and rotation; L = ext->L - 1.
he_status ks_check(const he_ctx* ext, uint64_t n) {
  if (check_ctx(ext)) return HE_EINVAL;
  if (ext->L < 2) return HE_EPARAM;
  const uint64_t L = ext->L - 1, per = ext->N / 256;
  if (n > ROT_MAX_BLOCKS / (L * (L + 1) * per)) return HE_ESHAPE;
  return HE_OK;
}

he_status ks_run(const he_ctx* ext, uint32_t ginv, uint64_t n, const uint64_t* ct, const uint64_t* ksk, uint64_t* out,
                 uint64_t* work, hipStream_t st, const uint64_t* addp = nullptr) {
  const uint32_t L = ext->L - 1, N = ext->N;
  const uint64_t P = ext->q[L];
  heconv::PinvConst pc{};
  for (uint32_t j = 0; j < L; j++) {
    const uint64_t q = ext->q[j];
    pc.v[j] = mpow(P % q, q - 2, q);
    pc.sh[j] = shoup(pc.v[j], q);
  }
  uint64_t* digits = work;                                   // [n][L][L+1][N]
  uint64_t* acc = work + n * L * (uint64_t)(L + 1) * N;      // [n][2][L+1][N]
  he_status s = HE_OK;
  const bool fusable = heconv::ks_fwd_supported(ext->logN);
  if (ext->tune.ks_fused == 1 && fusable) {
    s = dev_err(heconv::modup_ntt_launch(ext->logN, ct, digits, n, L, ginv, ext->d_fwd, ext->d_lc, st));
    if (!s) s = dev_err(heconv::inner_intt_launch(ext->logN, digits, ksk, acc, n, L, L, nullptr, nullptr, 0, 0, ext->d_inv,
                                                  ext->d_lc, st));
  } else {
    if (ext->tune.ks_fused == 2 && fusable) {
      s = dev_err(heconv::ks_fwd_launch(ext->logN, ct, ksk, acc, n, L, ginv, ext->d_fwd, ext->d_lc, st));
    } else {
      s = dev_err(heconv::modup_launch(ct, digits, n, N, L, ginv, ext->d_lc, st));
      if (!s) s = dev_err(ntt_run(ext, false, digits, n * L, st));
      if (!s) s = dev_err(heconv::ks_inner_launch(digits, ksk, acc, n, N, L, ext->d_lc, st));
    }
    if (!s) s = dev_err(ntt_run(ext, true, acc, 2 * n, st));
  }
  if (!s) s = dev_err(heconv::moddown_launch(acc, ct, out, n, N, L, ginv, pc, ext->d_lc, st, addp));
  return s;
}

}  // namespace

he_status he_keyswitch_work_words(const he_ctx* ext, uint64_t n, uint64_t* words) {
  if (!words) return HE_EINVAL;
  if (he_status s = ks_check(ext, n)) return s;
  const uint64_t L = ext->L - 1;
  *words = n * (L + 2) * (L + 1) * ext->N;
  return HE_OK;
}

he_status he_galois_key(const he_ctx* ext, uint64_t g, const int64_t* d_sk, const uint64_t* d_a, const int64_t* d_err,
                        uint64_t* d_ksk_ntt, uint64_t* d_work, void* stream) {
  if (check_ctx(ext)) return HE_EINVAL;
  if (ext->L < 2) return HE_EPARAM;
  if (!galois_ok(g, ext->N)) return HE_EINVAL;
  if (!d_sk || !d_a || !d_err || !d_ksk_ntt || !d_work) return HE_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const uint32_t L = ext->L - 1, L1 = ext->L, N = ext->N;
  const uint64_t LN1 = (uint64_t)L1 * N;
  uint64_t* w_a = d_work;               // [L][L+1][N]
  uint64_t* w_e = d_work + L * LN1;     // [L][L+1][N]
  uint64_t* w_s = d_work + 2 * L * LN1;  // [L+1][N], then s(X^g)
  he_status s = dev_err(hipMemcpyAsync(w_a, d_a, sizeof(uint64_t) * L * LN1, hipMemcpyDeviceToDevice, st));
  for (uint32_t l = 0; l < L && !s; l++)
    s = dev_err(heconv::key_lift_launch(d_err + (uint64_t)l * N, w_e + l * LN1, N, L1, ext->d_lc, st));
  if (!s) s = dev_err(heconv::key_lift_launch(d_sk, w_s, N, L1, ext->d_lc, st));
  if (!s) s = dev_err(heconv::automorph_launch(w_s, w_s + LN1, L1, N, L1, inv_mod_2n(g, N), ext->d_lc, st));
  if (!s) s = dev_err(ntt_run(ext, false, d_work, 2 * L + 2, st));
  if (!s) s = dev_err(heconv::galois_key_launch(d_work, d_ksk_ntt, N, L, ext->d_lc, st));
  return s;
}

he_status he_automorph(const he_ctx* c, uint64_t g, uint64_t n, const uint64_t* d_in, uint64_t* d_out, void* stream) {
  if (check_ctx(c)) return HE_EINVAL;
  if (!galois_ok(g, c->N)) return HE_EINVAL;
  if (n > ROT_MAX_BLOCKS / ((uint64_t)c->L * (c->N / 256))) return HE_ESHAPE;
  if (n == 0) return HE_OK;
  if (!d_in || !d_out || d_in == d_out) return HE_EINVAL;
  return dev_err(heconv::automorph_launch(d_in, d_out, n * c->L, c->N, c->L, inv_mod_2n(g, c->N), c->d_lc,
                                          (hipStream_t)stream));
}

he_status he_keyswitch(const he_ctx* ext, uint64_t n, const uint64_t* d_ct, const uint64_t* d_ksk_ntt, uint64_t* d_out,
                       uint64_t* d_work, void* stream) {
  if (he_status s = ks_check(ext, n)) return s;
  if (n == 0) return HE_OK;
  if (!d_ct || !d_ksk_ntt || !d_out || !d_work) return HE_EINVAL;
  return ks_run(ext, 1, n, d_ct, d_ksk_ntt, d_out, d_work, (hipStream_t)stream);
}

he_status he_zp_fold(const he_ctx* ext, uint64_t g, uint64_t n, const uint64_t* d_ct, const uint64_t* d_ksk_ntt,
                     uint64_t* d_out, uint64_t* d_work, void* stream) {
  if (he_status s = ks_check(ext, n)) return s;
  if (!galois_ok(g, ext->N)) return HE_EINVAL;
  if (n == 0) return HE_OK;
  if (!d_ct || !d_ksk_ntt || !d_out || !d_work || d_ct == d_out) return HE_EINVAL;
  return ks_run(ext, inv_mod_2n(g, ext->N), n, d_ct, d_ksk_ntt, d_out, d_work, (hipStream_t)stream, d_ct);
}

he_status he_rotate(const he_ctx* ext, uint64_t g, uint64_t n, const uint64_t* d_ct, const uint64_t* d_ksk_ntt,
                    uint64_t* d_out, uint64_t* d_work, void* stream) {
  if (he_status s = ks_check(ext, n)) return s;
  if (!galois_ok(g, ext->N)) return HE_EINVAL;
  if (n == 0) return HE_OK;
  if (!d_ct || !d_ksk_ntt || !d_out || !d_work || d_ct == d_out) return HE_EINVAL;
  return ks_run(ext, inv_mod_2n(g, ext->N), n, d_ct, d_ksk_ntt, d_out, d_work, (hipStream_t)stream);
}

// ---- Z_P variant: slots over a prime t, plaintexts, the linear kernel ----

namespace {

he_status t_ctx_check(const he_ctx* tc) {
  if (check_ctx(tc)) return HE_EINVAL;
  return tc->L == 1 ? HE_OK : HE_EPARAM;
}

}  // namespace

he_status he_simd_encode(const he_ctx* tctx, uint64_t n, const uint64_t* d_slots, int64_t* d_coeffs, void* stream) {
  if (he_status s = t_ctx_check(tctx)) return s;
  if (n == 0) return HE_OK;
  if (!d_slots || !d_coeffs || (const void*)d_slots == (const void*)d_coeffs) return HE_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  uint64_t* out = reinterpret_cast<uint64_t*>(d_coeffs);
  for (uint64_t i0 = 0; i0 < n; i0 += CLIENT_CHUNK) {
    const uint64_t m = n - i0 < CLIENT_CHUNK ? n - i0 : CLIENT_CHUNK;
    he_status s = dev_err(heconv::slot_permute_launch(d_slots + i0 * tctx->N, out + i0 * tctx->N, m, tctx->logN,
                                                      true, st));
    if (s) return s;
  }
  he_status s = dev_err(ntt_run(tctx, true, out, n, st));
  if (!s) s = dev_err(heconv::centre_launch(out, n * tctx->N, tctx->q[0], st));
  return s;
}

he_status he_simd_decode(const he_ctx* tctx, uint64_t n, const int64_t* d_coeffs, uint64_t* d_slots, uint64_t* d_work,
                         void* stream) {
  if (he_status s = t_ctx_check(tctx)) return s;
  if (n == 0) return HE_OK;
  if (!d_coeffs || !d_slots || !d_work || d_work == d_slots) return HE_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  he_status s = dev_err(heconv::reduce_t_launch(d_coeffs, d_work, n * tctx->N, tctx->lc[0], st));
  if (!s) s = dev_err(ntt_run(tctx, false, d_work, n, st));
  for (uint64_t i0 = 0; i0 < n && !s; i0 += CLIENT_CHUNK) {
    const uint64_t m = n - i0 < CLIENT_CHUNK ? n - i0 : CLIENT_CHUNK;
    s = dev_err(heconv::slot_permute_launch(d_work + i0 * tctx->N, d_slots + i0 * tctx->N, m, tctx->logN, false, st));
  }
  return s;
}

he_status he_zp_diagonals(const he_ctx* tctx, const int64_t* d_w, uint32_t rows, uint32_t cols, uint32_t n,
                          uint64_t* d_slots, void* stream) {
  if (he_status s = t_ctx_check(tctx)) return s;
  if (!pow2(n) || n > tctx->N / 2 || n > 65535 || rows == 0 || cols == 0 || rows > n || cols > n) return HE_ESHAPE;
  if (!d_w || !d_slots) return HE_EINVAL;
  return dev_err(heconv::diagonals_launch(d_w, rows, cols, n, n, tctx->N, d_slots, tctx->lc[0], (hipStream_t)stream));
}

he_status he_zp_diagonals_rect(const he_ctx* tctx, const int64_t* d_w, uint32_t rows, uint32_t cols, uint32_t n_out,
                               uint32_t n_in, uint64_t* d_slots, void* stream) {
  if (he_status s = t_ctx_check(tctx)) return s;
  if (!pow2(n_out) || !pow2(n_in) || n_out > n_in || n_in > tctx->N / 2 || n_out > 65535 || rows == 0 || cols == 0 ||
      rows > n_out || cols > n_in)
    return HE_ESHAPE;
  if (!d_w || !d_slots) return HE_EINVAL;
  return dev_err(heconv::diagonals_launch(d_w, rows, cols, n_out, n_in, tctx->N, d_slots, tctx->lc[0],
                                          (hipStream_t)stream));
}

he_status he_zp_encode_plain(const he_ctx* ext, uint64_t n, const int64_t* d_coeffs, uint64_t* d_w, void* stream) {
  if (check_ctx(ext)) return HE_EINVAL;
  if (ext->L < 2) return HE_EPARAM;
  if (n == 0) return HE_OK;
  if (!d_coeffs || !d_w) return HE_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const uint32_t L = ext->L - 1;
  const uint64_t P = ext->q[L];
  heconv::ScaleConst sc{};
  for (uint32_t l = 0; l < L; l++) {
    const uint64_t q = ext->q[l], pm = P % q;
    sc.v[l] = pm ? q - pm : 0;
    sc.sh[l] = shoup(sc.v[l], q);
  }
  for (uint64_t i0 = 0; i0 < n; i0 += CLIENT_CHUNK) {
    const uint64_t m = n - i0 < CLIENT_CHUNK ? n - i0 : CLIENT_CHUNK;
    he_status s = dev_err(heconv::lift_scaled_launch(d_coeffs + i0 * ext->N, d_w + i0 * L * ext->N, m, ext->N, L, sc,
                                                     ext->d_lc, st));
    if (s) return s;
  }
  return dev_err(heconv::ntt_launch(false, ext->logN, ntt_loge(ext, n), d_w, n, L, ext->d_fwd, ext->d_lc, st));
}

he_status he_zp_work_words(const he_ctx* ext, uint64_t n, uint64_t* words) {
  return he_zp_grouped_work_words(ext, n, 1, words);
}

he_status he_zp_grouped_work_words(const he_ctx* ext, uint64_t n, uint32_t groups, uint64_t* words) {
  if (!words || groups == 0) return HE_EINVAL;
  if (he_status s = ks_check(ext, n * groups)) return s;
  const uint64_t L = ext->L - 1, nc = n * groups;
  *words = 2 * nc * 2 * L * ext->N + nc * (L + 2) * (L + 1) * ext->N;
  return HE_OK;
}

namespace {

// The multiply-accumulate-rotate kernel as `groups` chains of n_diag/groups
// iterations (chain c takes diagonals c*per .. (c+1)*per - 1), run as one
// batch of groups*n ciphertexts, then acc = chain_{G-1} and
// acc = rotate(acc, g2) + chain_c for c = G-2 .. 0.
he_status zp_run(const he_ctx* ext, uint32_t g, uint64_t n, const uint64_t* d_x_ntt, const uint64_t* d_w,
                 uint32_t n_diag, uint32_t groups, const uint64_t* ksk, uint32_t g2, const uint64_t* ksk2,
                 uint64_t* d_out, uint64_t* d_work, hipStream_t st) {
  const uint32_t L = ext->L - 1, N = ext->N, ginv = inv_mod_2n(g, N);
  const uint64_t P = ext->q[L], ctw = 2ull * L * N;  // words per ciphertext
  heconv::PinvConst pc{};
  for (uint32_t j = 0; j < L; j++) {
    const uint64_t q = ext->q[j];
    pc.v[j] = mpow(P % q, q - 2, q);
    pc.sh[j] = shoup(pc.v[j], q);
  }
  const uint64_t nc = n * groups;
  const uint32_t per = n_diag / groups;
  // work: two accumulators of nc ciphertexts, digits [nc][L][L+1][N], sums
  // [nc][2][L+1][N].  The iterations depend on each other, so at a small
  // batch each runs at one workgroup's transform latency; running the
  // batch's two halves on two streams was measured slower (B = 16: 61.8
  // against 50.8 us per iteration), which is why chains are batched instead.
  uint64_t* accb[2] = {d_work, d_work + nc * ctw};
  uint64_t* digits = d_work + 2 * nc * ctw;
  uint64_t* sums = digits + nc * L * (uint64_t)(L + 1) * N;
  const uint64_t* prev = nullptr;  // the chains' accumulators (null: zero)
  uint32_t cur = 0;
  for (uint32_t step = 0; step < per; step++) {
    const uint32_t i = per - 1 - step;
    uint64_t* next = groups == 1 && step + 1 == per ? d_out : accb[cur];
    he_status s = HE_OK;
    if (prev) s = dev_err(heconv::modup_ntt_launch(ext->logN, prev, digits, nc, L, ginv, ext->d_fwd, ext->d_lc, st));
    if (!s)
      s = dev_err(heconv::inner_intt_launch(ext->logN, digits, ksk, sums, nc, L, prev ? L : 0, d_x_ntt,
                                            d_w + (uint64_t)i * L * N, n, (uint64_t)per * L * N, ext->d_inv,
                                            ext->d_lc, st));
    if (!s) s = dev_err(heconv::moddown_launch(sums, prev, next, nc, N, L, ginv, pc, ext->d_lc, st));
    if (s) return s;
    prev = next;
    cur ^= 1;
  }
  if (groups == 1) return HE_OK;
  // combine the chains: the other accumulator buffer holds two n-ciphertext
  // ping-pong slots (nc >= 2n)
  const uint32_t g2inv = inv_mod_2n(g2, N);
  uint64_t* tmp[2] = {accb[cur], accb[cur] + n * ctw};
  const uint64_t* acc = prev + (uint64_t)(groups - 1) * n * ctw;
  for (uint32_t c = groups - 1; c-- > 0;) {
    uint64_t* next = c == 0 ? d_out : tmp[c & 1];
    he_status s = dev_err(heconv::modup_ntt_launch(ext->logN, acc, digits, n, L, g2inv, ext->d_fwd, ext->d_lc, st));
    if (!s)
      s = dev_err(heconv::inner_intt_launch(ext->logN, digits, ksk2, sums, n, L, L, nullptr, nullptr, 0, 0,
                                            ext->d_inv, ext->d_lc, st));
    if (!s)
      s = dev_err(heconv::moddown_launch(sums, acc, next, n, N, L, g2inv, pc, ext->d_lc, st,
                                         prev + (uint64_t)c * n * ctw));
    if (s) return s;
    acc = next;
  }
  return HE_OK;
}

he_status zp_check(const he_ctx* ext, uint64_t g, uint64_t n, uint32_t n_diag, uint32_t groups) {
  if (he_status s = ks_check(ext, n * (groups ? groups : 1))) return s;
  if (!heconv::ks_fwd_supported(ext->logN)) return HE_EPARAM;
  if (!galois_ok(g, ext->N) || n_diag == 0 || groups == 0 || n_diag % groups) return HE_EINVAL;
  return HE_OK;
}

}  // namespace

he_status he_zp_matvec(const he_ctx* ext, uint64_t g, uint64_t n, const uint64_t* d_x_ntt, const uint64_t* d_w,
                       uint32_t n_diag, const uint64_t* d_ksk_ntt, uint64_t* d_out, uint64_t* d_work, void* stream) {
  if (he_status s = zp_check(ext, g, n, n_diag, 1)) return s;
  if (n == 0) return HE_OK;
  if (!d_x_ntt || !d_w || !d_ksk_ntt || !d_out || !d_work) return HE_EINVAL;
  return zp_run(ext, (uint32_t)g, n, d_x_ntt, d_w, n_diag, 1, d_ksk_ntt, 1, nullptr, d_out, d_work,
                (hipStream_t)stream);
}

he_status he_zp_matvec_grouped(const he_ctx* ext, uint64_t g, uint64_t n, const uint64_t* d_x_ntt, const uint64_t* d_w,
                               uint32_t n_diag, uint32_t groups, const uint64_t* d_ksk_ntt, uint64_t g2,
                               const uint64_t* d_ksk2_ntt, uint64_t* d_out, uint64_t* d_work, void* stream) {
  if (he_status s = zp_check(ext, g, n, n_diag, groups)) return s;
  if (groups > 1 && !galois_ok(g2, ext->N)) return HE_EINVAL;
  if (n == 0) return HE_OK;
  if (!d_x_ntt || !d_w || !d_ksk_ntt || !d_out || !d_work || (groups > 1 && !d_ksk2_ntt)) return HE_EINVAL;
  return zp_run(ext, (uint32_t)g, n, d_x_ntt, d_w, n_diag, groups, d_ksk_ntt, (uint32_t)g2, d_ksk2_ntt, d_out, d_work,
                (hipStream_t)stream);
}

// ---- polyphase form of strided convolutions ----

namespace {

bool poly_geom(const he_conv_desc* d, heconv::PolyGeom& g) {
  if (!d || d->stride < 2 || !d->C || !d->H || !d->W || !d->M || !d->kh || !d->kw) return false;
  const uint64_t s = d->stride, Cp = s * s * d->C;
  const uint64_t Hp = (d->H + 2ull * d->pad + s - 1) / s, Wp = (d->W + 2ull * d->pad + s - 1) / s;
  const uint64_t khp = (d->kh + s - 1) / s, kwp = (d->kw + s - 1) / s;
  if (Cp > 0xffffffffull || Hp < khp || Wp < kwp || d->H + 2ull * d->pad < d->kh || d->W + 2ull * d->pad < d->kw)
    return false;
  g = heconv::PolyGeom{d->C, d->H, d->W, d->M, d->kh, d->kw, d->stride, d->pad, (uint32_t)Cp, (uint32_t)Hp,
                       (uint32_t)Wp, (uint32_t)khp, (uint32_t)kwp};
  return true;
}

}  // namespace

he_status he_polyphase_desc(const he_conv_desc* in, he_conv_desc* out) {
  if (!in || !out) return HE_EINVAL;
  heconv::PolyGeom g;
  if (!poly_geom(in, g)) return HE_ESHAPE;
  *out = he_conv_desc{g.Cp, g.Hp, g.Wp, g.M, g.khp, g.kwp, 1, 0, 0, 0, 0};
  return HE_OK;
}

he_status he_polyphase_advised(uint32_t N, uint32_t L, const he_conv_desc* d, uint32_t batch_hint, int* use) {
  if (!d || !use) return HE_EINVAL;
  *use = 0;
  if (!batch_hint) batch_hint = 1;
  if (d->stride < 2) return HE_OK;
  he_conv_desc ds = *d, dp;
  ds.Cw = ds.Hw = ds.Ww = 0;
  if (he_status s = he_plan_conv_host(N, L, &ds, batch_hint)) return s;
  if (he_status s = he_polyphase_desc(d, &dp)) return s;
  if (he_status s = he_plan_conv_host(N, L, &dp, batch_hint)) return s;
  Geo gs, gp;
  if (!geo_of(ds, N, gs) || !geo_of(dp, N, gp)) return HE_ESHAPE;
  u128 bs, ms, bp, mp;
  plan_cost(ds, gs, N, L, batch_hint, bs, ms);
  plan_cost(dp, gp, N, L, batch_hint, bp, mp);
  *use = bp < bs || (bp == bs && mp < ms);
  return HE_OK;
}

he_status he_polyphase_weights(const he_conv_desc* d, const int64_t* d_w, int64_t* d_wp, void* stream) {
  heconv::PolyGeom g;
  if (!poly_geom(d, g)) return HE_ESHAPE;
  if (!d_w || !d_wp) return HE_EINVAL;
  return dev_err(heconv::polyphase_weights_launch(d_w, d_wp, g, (hipStream_t)stream));
}

he_status he_polyphase_input(const he_conv_desc* d, uint32_t B, const int64_t* d_x, int64_t* d_xp, void* stream) {
  heconv::PolyGeom g;
  if (!poly_geom(d, g)) return HE_ESHAPE;
  if (B == 0) return HE_OK;
  if (!d_x || !d_xp) return HE_EINVAL;
  return dev_err(heconv::polyphase_input_launch(d_x, d_xp, g, B, (hipStream_t)stream));
}

}  // extern "C"
