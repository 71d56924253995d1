// Internal launcher declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "modarith.h"

namespace heconv {

// One launch covers at most 2^32 - 1 work-items along x (workgroups times
// threads per workgroup): the largest grid of `threads`-thread workgroups.
constexpr uint64_t grid_max_blocks(uint32_t threads) { return 0xffffffffull / threads; }


// Forward (inverse = false) or inverse NTT, in place, of n_rns_polys RNS
// polynomials [n][L][N], N = 2^logN, logN in [10, 14]; 2^loge words per
// thread (loge 3 or 4; 3 needs logN <= 13, else 4 is used).  nt: the
// inverse transform stores its result non-temporally (a layer's output).
hipError_t ntt_launch(bool inverse, uint32_t logN, uint32_t loge, uint64_t* polys, uint64_t n_rns_polys, uint32_t L,
                      const Tw* tw, const LimbConst* lc, hipStream_t st, bool nt = false);

// Forward NTT in two grids (first six stages by residue class, the rest by
// block), for counts too small to occupy every compute unit; logN 12..14.
bool ntt_fwd_split_supported(uint32_t logN);
// the inverse in two grids (N = 2^13, 2^14)
bool ntt_inv_split_supported(uint32_t logN);
hipError_t ntt_inv_split_launch(uint32_t logN, uint64_t* polys, uint64_t n_rns_polys, uint32_t L, const Tw* tw,
                                const LimbConst* lc, hipStream_t st);
hipError_t ntt_fwd_split_launch(uint32_t logN, uint64_t* polys, uint64_t n_rns_polys, uint32_t L, const Tw* tw,
                                const LimbConst* lc, hipStream_t st);

// NTT / inverse NTT in double precision (every q_l < 2^50): tw are the
// twiddles as doubles ([L][N], forward or inverse table), fc the per-limb
// constants filled by f64_const_fill (f64_const_size bytes each).
size_t f64_const_size();
void f64_const_fill(void* out, double q, double qinv, double ninv, double ninv_w);
hipError_t ntt_f64_launch(bool inverse, uint32_t logN, uint32_t loge, uint64_t* polys, uint64_t n_rns_polys,
                          uint32_t L, const double* tw, const void* fc, hipStream_t st);

// Rotation (automorphism + hybrid key switching with a special prime).
struct PinvConst {
  uint64_t v[7], sh[7];  // P^-1 mod q_j and its Shoup quotient, j < L (L <= 7)
};
hipError_t automorph_launch(const uint64_t* in, uint64_t* out, uint64_t rows, uint32_t N, uint32_t L, uint32_t ginv,
                            const LimbConst* lc, hipStream_t st);
hipError_t modup_launch(const uint64_t* ct, uint64_t* work, uint64_t n, uint32_t N, uint32_t L, uint32_t ginv,
                        const LimbConst* ext, hipStream_t st);
hipError_t ks_inner_launch(const uint64_t* work, const uint64_t* ksk, uint64_t* acc, uint64_t n, uint32_t N,
                           uint32_t L, const LimbConst* ext, hipStream_t st);
hipError_t moddown_launch(const uint64_t* acc, const uint64_t* ct, uint64_t* out, uint64_t n, uint32_t N, uint32_t L,
                          uint32_t ginv, const PinvConst& pinv, const LimbConst* ext, hipStream_t st,
                          const uint64_t* addp = nullptr);
bool ks_fwd_supported(uint32_t logN);
hipError_t ks_fwd_launch(uint32_t logN, const uint64_t* ct, const uint64_t* ksk, uint64_t* acc, uint64_t n, uint32_t L,
                         uint32_t ginv, const Tw* tw, const LimbConst* ext, hipStream_t st);
hipError_t modup_ntt_launch(uint32_t logN, const uint64_t* ct, uint64_t* digits, uint64_t n, uint32_t L, uint32_t ginv,
                            const Tw* tw, const LimbConst* ext, hipStream_t st);
hipError_t inner_intt_launch(uint32_t logN, const uint64_t* digits, const uint64_t* ksk, uint64_t* acc, uint64_t n,
                             uint32_t L, uint32_t nd, const uint64_t* xp, const uint64_t* wp, uint64_t chain_cts,
                             uint64_t w_stride, const Tw* tw_inv, const LimbConst* ext, hipStream_t st);
hipError_t galois_key_launch(const uint64_t* work, uint64_t* ksk, uint32_t N, uint32_t L, const LimbConst* ext,
                             hipStream_t st);

// Z_P variant: slots, diagonals, scaled plaintext lift.
struct ScaleConst {
  uint64_t v[7], sh[7];  // a per-limb factor mod q_l and its Shoup quotient
};
hipError_t slot_permute_launch(const uint64_t* in, uint64_t* out, uint64_t n, uint32_t logN, bool encode,
                               hipStream_t st);
hipError_t centre_launch(uint64_t* v, uint64_t words, uint64_t t, hipStream_t st);
hipError_t reduce_t_launch(const int64_t* in, uint64_t* out, uint64_t words, const LimbConst& tc, hipStream_t st);
hipError_t diagonals_launch(const int64_t* W, uint32_t rows, uint32_t cols, uint32_t n_out, uint32_t n_in, uint32_t N,
                            uint64_t* slots, const LimbConst& tc, hipStream_t st);
hipError_t lift_scaled_launch(const int64_t* c, uint64_t* out, uint64_t n, uint32_t N, uint32_t L,
                              const ScaleConst& sc, const LimbConst* lc, hipStream_t st);

// Polyphase form of a strided conv: the original (C, H, W, M, kh, kw, s,
// pad) and the phase conv's channels, size and kernel.
struct PolyGeom {
  uint32_t C, H, W, M, kh, kw, s, pad, Cp, Hp, Wp, khp, kwp;
};
hipError_t polyphase_weights_launch(const int64_t* K, int64_t* Kp, const PolyGeom& g, hipStream_t st);
hipError_t polyphase_input_launch(const int64_t* x, int64_t* X, const PolyGeom& g, uint64_t B, hipStream_t st);

// Geometry of a planned conv as the kernels need it.
struct PackGeom {
  uint32_t M, C, kh, kw, Cw, Hw, Ww, CB, L, N, O;
};

// Kernel polynomials in coefficient form: out[M][CB][L][N], lifted mod q_l.
hipError_t pack_weights_launch(const PackGeom& g, const int64_t* w, uint64_t* out, const LimbConst* lc,
                               hipStream_t st);

// out[b][m][s][c][l][k] = sum_cb in[b][cb][s][c][l][k] * w[m][cb][l][k] mod q_l.
// (mt, rt): output channels x rows per thread; (0, 0), or a pair the chosen
// kernel is not built for, picks by shape.  lds_stages: 0 = operands loaded
// into registers (mac_tile), 2..4 = the streamed MAC (mac_stream) staging
// them in LDS that many channel blocks ahead, for layers whose weight pairs
// fit 32-bit offsets (others take the register loads).  all_pm: every q_l is
// 2^60 - delta, delta < 2^20 (the streamed MAC's short fold).  grid: the
// streamed MAC runs each workgroup's four waves as a 2x2 grid (tiles of
// 2*mt channels x 2*rt rows, mac_grid.h) when the layer has that many rows
// and channels.
hipError_t mac_launch(const uint64_t* in, const uint64_t* w, uint64_t* out, uint32_t B, uint32_t CB, uint32_t S,
                      uint32_t M, uint32_t L, uint32_t N, const LimbConst* lc, uint32_t mt, uint32_t rt,
                      uint32_t lds_stages, bool all_pm, bool grid, hipStream_t st);

// Whether the LDS-staged MAC can take a layer: two output channels' weights
// (2*CB*L*N words) below 2^31 bytes.
inline bool mac_dma_fits(uint32_t CB, uint32_t L, uint32_t N) {
  return (uint64_t)2 * CB * L * N * 8 < (1ull << 31);
}

// Fused MAC + inverse NTT: in (NTT form) x w -> out (coefficient form).
hipError_t mac_intt_launch(uint32_t logN, const uint64_t* in, const uint64_t* w, uint64_t* out, uint32_t B,
                           uint32_t CB, uint32_t S, uint32_t M, uint32_t L, const Tw* twi, const LimbConst* lc,
                           hipStream_t st);

// Geometry of the protocol steps around a layer (conv, packing, tiling).
struct ProtoGeom {
  uint32_t B, C, H, W, M, Cw, Hw, Ww;
  uint32_t bh, bw, nsj, S, CB, O, He, We, Ho, Wo;
  uint32_t step;   // stride of the packed tensor's rows/columns in the padded input (strided 1x1: stride, else 1)
  uint32_t ostep;  // stride-1 output rows/columns per kept output (1 for a strided 1x1 conv, else stride)
  int32_t pad;
  uint32_t L, N;
  uint64_t t;
};

// b_l += delta_l * pack(share) mod q_l for in [B][CB][S][2][L][N], share
// [B][C][H][W] (values taken mod t).
hipError_t add_share_launch(uint64_t* in, const int64_t* share, const ProtoGeom& g, const LimbConst* lc,
                            hipStream_t st);

// y[b][m][l][oy][ox] = b-coefficient of output (oy, ox) - delta_l * mask + noise mod q_l.
hipError_t mask_extract_launch(const uint64_t* out, const int64_t* mask, const int64_t* noise, uint64_t* y,
                               const ProtoGeom& g, const LimbConst* lc, hipStream_t st);

// Client-side decoding constants of one limb: with y_l = (Q/q_l)^-1 mod q_l,
// ipart = floor(t*y_l/q_l) and (frac_hi, frac_lo) = floor(frac(t*y_l/q_l) * 2^128).
struct DecodeConst {
  uint64_t ipart, frac_hi, frac_lo;
};

// Client-side steps (secret key on the device): key lift, copy of the a
// components, point-wise product with the transformed key, encryption and
// decryption finish.  n <= 65535 RNS polynomials per call.
hipError_t key_lift_launch(const int64_t* sk, uint64_t* out, uint32_t N, uint32_t L, const LimbConst* lc,
                           hipStream_t st);
hipError_t copy_a_launch(const uint64_t* src, uint64_t src_stride, uint64_t* work, uint64_t* ct_out, uint64_t n,
                         uint32_t N, uint32_t L, hipStream_t st);
hipError_t pointwise_key_launch(uint64_t* work, const uint64_t* sk_ntt, uint64_t n, uint32_t N, uint32_t L,
                                const LimbConst* lc, hipStream_t st);
hipError_t encrypt_finish_launch(const uint64_t* as, const int64_t* msg, const int64_t* err, uint64_t* ct, uint64_t n,
                                 uint32_t N, uint32_t L, uint64_t t, const LimbConst* lc, hipStream_t st);
hipError_t decrypt_finish_launch(const uint64_t* ct, const uint64_t* as, int64_t* out, uint64_t n, uint32_t N,
                                 uint32_t L, const LimbConst& tc, const DecodeConst* dc, const LimbConst* lc,
                                 hipStream_t st);

}  // namespace heconv
