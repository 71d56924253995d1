/*
 * heconv.h -- C ABI of the MI355X (gfx950) homomorphic-convolution library.
 *
 * The server side of an HE convolution on RNS BFV ciphertexts, as the paper
 * describes it (SecONNds, arXiv 2506.11586, Sec. 6.2 "NTT preprocessing"):
 * weights are encoded and NTT-transformed once; each incoming ciphertext is
 * NTT-transformed on receipt; every multiply-accumulate runs in the NTT
 * domain, summed over input-channel blocks; only the final results are
 * inverse-transformed.  The library never handles key material (Sec. 6.3:
 * the GPU side computes only on encrypted data).
 *
 * Conventions for every entry point:
 *  - All functions return he_status; nothing throws across the ABI.
 *  - Pointers named d_* are device pointers (HIP device memory on the
 *    device that was current when the context was created).  The caller
 *    owns every buffer; the library owns only its context tables.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Work is
 *    enqueued asynchronously; errors raised by asynchronous work surface as
 *    HE_EDEVICE from a later call or from the caller's synchronisation.
 *  - Ciphertext and plaintext words are uint64 residues.  Inputs must be
 *    canonical (< q_l of their limb); outputs are always canonical.
 *  - An RNS polynomial is [L][N] words, limb-major: limb l holds the N
 *    coefficients (or NTT values) modulo q_l.  A ciphertext is two RNS
 *    polynomials (a, b) in the paper's order (App. C): component 0 = a,
 *    component 1 = b.
 *  - NTT form: entry i of a limb is the evaluation of the polynomial at
 *    psi_l^(2*brv(i)+1), brv = bit reversal over log2 N bits, psi_l the
 *    smallest primitive 2N-th root of unity mod q_l (App. C.1).
 *  - No entry point allocates device memory except he_ctx_create and
 *    he_batch_create.
 */
#ifndef HECONV_H
#define HECONV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HE_OK = 0,
  HE_EINVAL = -1,  /* null pointer, zero-sized descriptor field, bad flag */
  HE_ESHAPE = -2,  /* packing descriptor does not fit N or the layer */
  HE_EPARAM = -3,  /* unsupported N, q not prime / not 1 mod 2N / too large */
  HE_ENOMEM = -4,  /* device allocation failed (context creation only) */
  HE_EDEVICE = -5, /* a HIP call or kernel launch failed */
  HE_EBUSY = -6    /* reserved */
} he_status;

/* BFV/RNS parameters.  N: ring degree, a power of two in [2^10, 2^14].
 * L: number of RNS limbs, 1..8.  q[0..L-1]: distinct primes, q_l = 1 mod 2N,
 * 2^30 < q_l < 2^60 (the MAC splits residues into 30-bit halves).
 * t: plaintext modulus.  The layer path does not depend on it; the protocol
 * steps (he_add_share, he_mask_extract) need 2 <= t <= 2^62 and t < Q and
 * return HE_EPARAM otherwise. */
typedef struct {
  uint32_t N, L;
  const uint64_t* q;
  uint64_t t;
} he_params;

/* One convolution layer (cross-correlation as in CNNs): input C x H x W,
 * M output channels, kh x kw kernel, stride, zero padding `pad` on every
 * side.  (Cw, Hw, Ww) is the packing descriptor: Cw channels of an Hw x Ww
 * window per ciphertext (Cw*Hw*Ww <= N).  A strided conv with a kernel
 * larger than 1x1 is evaluated at stride 1 (the client keeps every
 * stride-th output); a strided 1x1 conv expects the client to subsample the
 * padded input first.  The packing layout is:
 *   input poly (channel block cb, tile s): coeff cc*Hw*Ww + i*Ww + j
 *     = padded input[cb*Cw+cc][si*bh+i][sj*bw+j], bh = Hw-kh+1, bw = Ww-kw+1
 *   kernel poly (m, cb): coeff O - cc*Hw*Ww - i*Ww - j = K[m][cb*Cw+cc][i][j],
 *     O = (Cw-1)*Hw*Ww + (kh-1)*Ww + (kw-1)
 *   output (m, tile s): coeff O + i*Ww + j = stride-1 output at
 *     (si*bh+i, sj*bw+j), i < bh, j < bw.
 * The paper gives no formula for this coefficient encoding (Sec. 6.1 and
 * Sec. 2.3, Cheetah paragraph); this layout is the library's. */
typedef struct {
  uint32_t C, H, W, M, kh, kw, stride, pad;
  uint32_t Cw, Hw, Ww;
} he_conv_desc;

typedef struct he_ctx he_ctx;

/* Status as text (static string). */
const char* he_status_str(he_status s);

/* The L largest primes below 2^bits that are 1 mod 2N, in descending order,
 * written to q_out[0..L-1].  HE_EPARAM if N is not a power of two, bits is
 * outside [20, 60], or fewer than L such primes exist. */
he_status he_gen_primes(uint32_t N, uint32_t bits, uint32_t L, uint64_t* q_out);

/* Create a context on the current HIP device (the ring Z_Q[X]/(X^N+1) of
 * Sec. 2.1 in RNS form, App. C): checks the parameters, picks
 * psi_l (the smallest primitive 2N-th root of unity mod q_l), builds the
 * twiddle tables (powers of psi in bit-reversed order with their Shoup
 * quotients, N^-1) and copies them to the device.  *out receives the
 * context; destroy it with he_ctx_destroy. */
he_status he_ctx_create(const he_params* prm, he_ctx** out);
void he_ctx_destroy(he_ctx* ctx);

/* Launch-shape choices of a context (they change speed, never results).
 * NTT: 2^ntt_loge_small words per thread (one workgroup of N/2^loge
 * threads per limb polynomial) when a call transforms fewer than
 * ntt_small_below limb polynomials, else 2^ntt_loge_large; loge is 3 or 4
 * (3 is used only for N <= 2^13).  MAC: each thread accumulates mac_mt
 * output channels x mac_rt ciphertext rows for one NTT point; (0, 0) picks
 * by shape; supported pairs: (4,4) (4,2) (2,4) (8,2) (2,8) (8,1) (1,8) (2,2),
 * and for batches with the streamed MAC (mac_lds 2-4) also (6,4) (8,4)
 * (4,8), which he_conv_ntt_mac and he_conv_layer replace by the shape's
 * default.  A batch takes the context's pair when its MAC is built for it
 * (streamed: (4,4) (6,4) (8,4) (4,8) (4,2) (2,4) (2,2); register loads:
 * (4,4) (4,2) (2,4) (2,2)); else (2,2) when a job has fewer than four
 * output channels, (4,2) when a job has fewer than four ciphertext rows,
 * else (4,4) on the 2x2 wave grid (mac_grid) when every
 * job has at least 8 rows and output channels, else (6,4) for the streamed
 * MAC when every job has at least six output channels, else (4,4).
 * layer_fused: 1 = he_conv_layer runs the MAC and the inverse NTT as one
 * kernel (he_conv_mac_intt), 0 = as two (he_conv_ntt_mac, he_ntt_inv).
 * (the fused kernel gives up the MAC's register tiling, so it moves several
 * times more data through L2 and is slower on the 64->64 3x3 layer: 153 us
 * against 106 us for the pair).
 * layer_split: 1, 2 or 4.  For one image (B = 1, M >= 8*split) he_conv_layer
 * cuts the output channels into that many slices: their MACs run in order
 * on the caller's stream, and the inverse NTT of each slice runs on the
 * context's internal stream once its MAC is done, beside the next slice's
 * MAC; the caller's stream then waits for the last transform.  The internal
 * stream is shared by all calls on the context: concurrent calls on several
 * streams should use 1.
 * ntt_split_below: he_ntt_fwd (and so he_conv_layer's forward step) runs
 * the forward NTT of fewer than this many limb polynomials (N = 2^12 ..
 * 2^14) as two grids of 128-thread workgroups, eight per 2^13 points,
 * instead of one workgroup per polynomial, so that every compute unit
 * takes part; 0 = never.  Measured at N = 2^13: 10.2 against 14.2 us for 48
 * limb polynomials, 11.2 against 14.9 for 96, 14.5 against 15.3 for 144,
 * but 16.9 against 15.6 for 192.
 * ntt_fp64: 1 = when every q_l < 2^50, every transform of the library
 * (except the batch executor's and the fused kernel's) runs in double
 * precision: residues are exact doubles and a modular product is two
 * products, two fused multiply-adds, a rounding and a conditional add, all
 * at the full fp64 rate, where the integer path's 32-bit multiplies run at
 * half rate.  0 = always the integer kernels.
 * ks_fused: how key switching and rotation (N <= 2^13) run their steps.
 * 1 = two fused kernels: digit extension (and the automorphism) in the
 * forward transform's load, the inner product with the key in the inverse
 * transform's load.  2 = one kernel extends, transforms and multiplies all
 * digits of a (ciphertext, modulus) pair by the key and stores only the two
 * sums (registers limit it to one workgroup per compute unit).  0 = the
 * steps as separate kernels.  Results are the same words in every mode.
 * ntt_inv_split_below: inverse NTTs of fewer than this many limb
 * polynomials (N = 2^13 and 2^14) run as two grids of 128-thread
 * workgroups, eight per 2^13 points (the stages on the low bits in blocks of
 * 2^(n-6) consecutive entries, then the top six stages per residue); 0 =
 * never.  Measured at N = 2^13: 9.5-11.0 against 13.0-13.9 us for 3 to 96
 * limb polynomials, 14.4 against 14.2 for 144, 16.8 against 14.8 for 192.
 * At N = 2^12 one workgroup per polynomial was faster at every count (7.5
 * against 9.7 us), so that size never splits.
 * mac_lds: 0 = the MAC loads its operands into registers, 4 channel
 * blocks at a time; 2, 3 or 4 = each wave stages its operands in a private
 * LDS ring that many channel blocks ahead with direct buffer-to-LDS loads,
 * so the loads in flight hold no registers (tiles with even mac_mt and
 * mac_rt, and layers whose two output channels' weights stay below 2^31
 * bytes; others keep the register loads).  Used by he_conv_ntt_mac,
 * he_conv_layer and batches created after it is set; in a batch it selects
 * the streamed MAC: each workgroup runs mac_tiles tiles (0 = 4) decoded on
 * the host, its loads running ahead across tile boundaries, with three
 * accumulators per output (a fold every 8 channel blocks).  Measured with
 * the 4x4 tile: three stages take the 64->64 3x3 layer's MAC from 71 to
 * 57 us with the caches flushed (46.8 to 43.9 us warm) and the 16-image
 * bottleneck CNN's MAC grid from 129.6 to 121.1 ms.
 * mac_tiles: tiles per workgroup of a batch's streamed MAC (0 = 4, at most
 * 64).
 * mac_grid: 1 (default) = the streamed MAC (a batch's, and that of
 * he_conv_ntt_mac and he_conv_layer) runs its workgroup's four waves as a
 * 2x2 grid over one slice of 64 NTT points, sharing the input and weight
 * rows they load (tiles of 2*mac_mt channels x 2*mac_rt rows, one workgroup
 * barrier per channel block), when every job (the layer) has that many rows
 * and channels; 0 = each wave its own 64 points.  Measured on the 16-image
 * bottleneck CNN's MAC grid: 98 ms per wave (6x4 tiles), 90 ms on the grid
 * (4x4 per wave, three stages), 88 ms with four stages.
 * Defaults: {3, 3, 512, 0, 0, 0, 1, 160, 1, 1, 128, 3, 0, 1}: 8 words per thread was measured faster
 * than 16 at every count at N = 8192 (768 limb polys: 47.7 against 51.4 us
 * inverse); N = 16384 always uses 16.  The channel pipeline (layer_split)
 * was measured slower than the plain order on 64->64, 128->128 and
 * 256->256 3x3 layers (141 / 153 us against 127 us on 64->64): the MAC and
 * the transforms compete for the same compute units instead of
 * overlapping. */
typedef struct {
  uint32_t ntt_loge_small, ntt_loge_large, ntt_small_below;
  uint32_t mac_mt, mac_rt;
  uint32_t layer_fused;
  uint32_t layer_split;
  uint32_t ntt_split_below;
  uint32_t ntt_fp64;
  uint32_t ks_fused;
  uint32_t ntt_inv_split_below;
  uint32_t mac_lds;
  uint32_t mac_tiles;
  uint32_t mac_grid;
} he_tuning;

he_status he_ctx_get_tuning(const he_ctx* ctx, he_tuning* out);
/* HE_EINVAL for an unsupported value; the context is then unchanged. */
he_status he_ctx_set_tuning(he_ctx* ctx, const he_tuning* tuning);

/* The roots chosen by the context: psi_out[0..L-1]. */
he_status he_ctx_psi(const he_ctx* ctx, uint64_t* psi_out);

/* Packing descriptor by exhaustive search (the library's planner): every
 * Hw in [kh, He], Ww in [kw, We] with Hw*Ww <= N (He x We = padded input,
 * subsampled for a strided 1x1 conv), Cw = min(C, N / (Hw*Ww)); minimise
 * the unfused HBM bytes M*CB*L*N*8 + batch*3*(in_cts+out_cts)*2*L*N*8, then
 * the modmul count, then prefer larger Hw, then larger Ww.  Fills io->Cw,
 * io->Hw, io->Ww.  batch_hint = number of images a launch will carry. */
he_status he_plan_conv(const he_ctx* ctx, he_conv_desc* io, uint32_t batch_hint);

/* The same planner without a context (host only, no device needed):
 * N a power of two, L >= 1. */
he_status he_plan_conv_host(uint32_t N, uint32_t L, he_conv_desc* io, uint32_t batch_hint);

/* The root a context would pick for (q, N): the smallest primitive 2N-th
 * root of unity mod q (host only).  HE_EPARAM unless q is a prime below
 * 2^62 with q = 1 mod 2N. */
he_status he_min_root(uint64_t q, uint32_t N, uint64_t* psi_out);

/* Sizes for a planned layer (per image; the ciphertext counts of the
 * coefficient encoding of Sec. 6.1 under the layout above): CB = ceil(C/Cw) channel blocks,
 * S spatial tiles, in_cts = CB*S, out_cts = M*S, w_words = M*CB*L*N.  Any
 * output pointer may be NULL.  HE_ESHAPE if the descriptor is invalid. */
he_status he_conv_sizes(const he_ctx* ctx, const he_conv_desc* desc, uint32_t* CB, uint32_t* S,
                        uint64_t* in_cts, uint64_t* out_cts, uint64_t* w_words);

/* Offline step: NTT preprocessing of the weights (Sec. 6.2).  Packs
 * d_w[M][C][kh][kw] (signed int64, device) into kernel polynomials, lifts
 * each signed value into [0, q_l), and forward-NTTs every limb.
 * d_wntt: [M][CB][L][N] uint64, written completely. */
he_status he_encode_weights(const he_ctx* ctx, const he_conv_desc* desc, const int64_t* d_w, uint64_t* d_wntt,
                            void* stream);

/* Forward negacyclic NTT, in place, of n RNS polynomials d_polys[n][L][N]
 * (App. C.1).  n = 0 is a no-op. */
he_status he_ntt_fwd(const he_ctx* ctx, uint64_t* d_polys, uint64_t n, void* stream);

/* Inverse NTT, in place (App. C.1; Sec. 6.2: only the final results leave
 * the NTT domain): d_polys[n][L][N] from NTT form back to
 * coefficients (including the factor N^-1).  The input is read and the
 * result written non-temporally (streamed past the caches: a layer's MAC
 * output is read once and its result not again soon), as he_conv_ntt_mac
 * writes its output. */
he_status he_ntt_inv(const he_ctx* ctx, uint64_t* d_polys, uint64_t n, void* stream);

/* Multiply-accumulate in the NTT domain over channel blocks (Sec. 6.2):
 *   out[b][m][s][c][l][k] = sum_{cb<CB} in[b][cb][s][c][l][k] * w[m][cb][l][k] mod q_l
 * d_in_ntt: [B][CB][S][2][L][N], d_wntt: [M][CB][L][N],
 * d_out_ntt: [B][M][S][2][L][N] (written completely; must not alias the
 * inputs).  HE_ESHAPE if one image's input ciphertexts (CB*S*2*L*N words)
 * or one output channel's weights (CB*L*N words) reach 2^31 bytes: the MAC
 * addresses them with 32-bit offsets (he_conv_layer and he_batch_create
 * check the same). */
he_status he_conv_ntt_mac(const he_ctx* ctx, const he_conv_desc* desc, uint32_t B, const uint64_t* d_in_ntt,
                          const uint64_t* d_wntt, uint64_t* d_out_ntt, void* stream);

/* The MAC and the inverse NTT in one kernel: from NTT-form inputs
 * d_in_ntt [B][CB][S][2][L][N] and weights to coefficient-form outputs
 * d_out [B][M][S][2][L][N] -- the same words as he_conv_ntt_mac followed by
 * he_ntt_inv, without the NTT-form output passing through HBM (Sec. 6.2: all
 * MACs in the NTT domain, only final results transformed back). */
he_status he_conv_mac_intt(const he_ctx* ctx, const he_conv_desc* desc, uint32_t B, const uint64_t* d_in_ntt,
                           const uint64_t* d_wntt, uint64_t* d_out, void* stream);

/* The whole online layer (Sec. 6.2, NTT preprocessing: inputs transformed
 * on receipt, every MAC in the NTT domain, results transformed back):
 * forward NTT of the B*CB*S input ciphertexts in
 * place (d_in is clobbered: it holds their NTT form afterwards), the MAC,
 * then the inverse NTT of the B*M*S output ciphertexts.
 * d_in: [B][CB][S][2][L][N] coefficient form; d_out: [B][M][S][2][L][N]
 * coefficient form. */
he_status he_conv_layer(const he_ctx* ctx, const he_conv_desc* desc, uint32_t B, uint64_t* d_in,
                        const uint64_t* d_wntt, uint64_t* d_out, void* stream);

/* ------------------------------------------------------------------------
 * Protocol steps either side of the layer (Sec. 7, online protocol for a
 * linear layer: the server adds its share of the input to the client's
 * ciphertexts, runs the layer on NTT-preprocessed weights, masks the result;
 * Sec. 6.2: only the coefficients that hold outputs are extracted).
 * delta_l = floor(Q/t) mod q_l, Q = q_0 * ... * q_{L-1}.
 * ------------------------------------------------------------------------ */

/* delta_l for L moduli q[0..L-1] (host only, no device needed):
 * HE_EPARAM if t is outside [2, 2^62] or exceeds Q (or some delta_l is 0). */
he_status he_delta_host(const uint64_t* q, uint32_t L, uint64_t t, uint64_t* delta_out);

/* Fold the server's additive share of the layer input into the client's
 * input ciphertexts, before he_conv_layer: with m = the share packed as the
 * layout above packs an input (values taken mod t, zero outside the
 * tensor), b_l <- b_l + delta_l * m mod q_l for every ciphertext; the a
 * components are untouched.  The result decrypts to (client share + server
 * share) mod t.
 * d_in: [B][CB][S][2][L][N] coefficient form, canonical, updated in place.
 * d_share: int64 [B][C][H][W] (unpadded; any values, reduced mod t).
 * HE_EPARAM if the context's t is unusable; B = 0 is a no-op. */
he_status he_add_share(const he_ctx* ctx, const he_conv_desc* desc, uint32_t B, uint64_t* d_in,
                       const int64_t* d_share, void* stream);

/* Mask and extract the outputs, after he_conv_layer: for every output
 * position (oy, ox) at the layer's stride (Ho = (H+2*pad-kh)/stride + 1,
 * Wo likewise) take the b coefficient that holds it (tile and index as in
 * the layout above; stride-1 position (oy*stride, ox*stride), or (oy, ox)
 * for a strided 1x1 conv), and write
 *   y[b][m][l][oy][ox] = b_l - delta_l * (mask mod t) + noise mod q_l.
 * The mask is the server's output share (the client decrypts conv - mask
 * mod t); noise is an optional signed smudging term per output (NULL = 0).
 * The random values are drawn by the caller.  The a components of d_out
 * are what the client needs besides y; they are not copied.
 * d_out: [B][M][S][2][L][N] coefficient form (read only).
 * d_mask, d_noise: int64 [B][M][Ho][Wo].  d_y: uint64 [B][M][L][Ho][Wo],
 * written completely, canonical.
 * HE_EPARAM if the context's t is unusable; B = 0 is a no-op. */
he_status he_mask_extract(const he_ctx* ctx, const he_conv_desc* desc, uint32_t B, const uint64_t* d_out,
                          const int64_t* d_mask, const int64_t* d_noise, uint64_t* d_y, void* stream);

/* ------------------------------------------------------------------------
 * Client side on the GPU (App. C, symmetric-key BFV): encryption of
 * coefficient-encoded messages and decryption, for load generation and for
 * checking results.  These calls take the secret key; the server-side calls
 * above never do.  Random values (a, e) are drawn by the caller.
 * ------------------------------------------------------------------------ */

/* The secret key in NTT form: d_sk_ntt[l][k] = NTT_l(sk mod q_l), from the
 * key's N integer coefficients d_sk (int64, normally in {-1, 0, 1}). */
he_status he_key_encode(const he_ctx* ctx, const int64_t* d_sk, uint64_t* d_sk_ntt, void* stream);

/* Encrypt n messages: for each i and limb l,
 *   ct[i][0][l] = a[i][l],  ct[i][1][l] = a[i][l]*sk + delta_l*(m[i] mod t) + e[i]  (mod q_l),
 * products in Z_q[X]/(X^N+1).  d_msgs, d_err: int64 [n][N]; d_a: [n][L][N]
 * canonical; d_sk_ntt from he_key_encode; d_ct: [n][2][L][N] written
 * completely; d_work: [n][L][N] caller-provided scratch (clobbered).
 * HE_EPARAM if the context's t is unusable; n = 0 is a no-op. */
he_status he_encrypt(const he_ctx* ctx, uint64_t n, const int64_t* d_msgs, const uint64_t* d_a,
                     const int64_t* d_err, const uint64_t* d_sk_ntt, uint64_t* d_ct, uint64_t* d_work,
                     void* stream);

/* Decrypt n ciphertexts [n][2][L][N]: v = b - a*sk per limb, then
 * m = round(t*V/Q) mod t for V the CRT lift of v, centred into
 * [-t/2, t/2), written to d_msgs (int64 [n][N]).  The rounding is computed
 * from fixed-point constants (128-bit fractions, total error below
 * L * 2^-68); it equals exact rounding whenever t*V/Q is not within that of
 * a half-integer, which holds for every ciphertext whose noise is below
 * delta/2 by a margin of a few units.  Any t with 2 <= t < 2^62 (a power
 * of two, or the prime plaintext modulus of the Z_P variant; for odd t the
 * range is -(t-1)/2 .. (t-1)/2), HE_EPARAM otherwise.  d_work: [n][L][N]
 * scratch. */
he_status he_decrypt(const he_ctx* ctx, uint64_t n, const uint64_t* d_ct, const uint64_t* d_sk_ntt, int64_t* d_msgs,
                     uint64_t* d_work, void* stream);

/* ------------------------------------------------------------------------
 * Rotation for the Z_P variant (Sec. 2: a rotation is a Galois automorphism
 * followed by key switching with an evaluation key; Sec. 6.1: the Z_P
 * kernels rotate once per multiply-accumulate iteration).  Key switching is
 * hybrid RNS key switching with one special prime P: the calls take an
 * EXTENDED context created with the L ciphertext primes followed by P
 * (ext->L = L + 1; P distinct and of about the size of the q's, which keeps
 * the added noise near N*L*q*e/P).  Ciphertexts are [n][2][L][N] in
 * coefficient form, canonical, of phase b - a*s.
 * Key layout (d_ksk_ntt): [L][2][L+1][N] residues over q_0..q_{L-1}, P in
 * NTT form (transform coefficient-form keys with he_ntt_fwd on the extended
 * context, 2L RNS polynomials): for digit l the pair (k_a, k_b) with
 * k_b = k_a*s + e_l + G_l*s' over Z_QP, G_l = P * Qhat_l * (Qhat_l^-1 mod q_l)
 * and Qhat_l = Q/q_l, which switches from s' to s.  The caller makes keys.
 * ------------------------------------------------------------------------ */

/* Words of scratch that he_keyswitch and he_rotate need for n ciphertexts:
 * n * (L+2) * (L+1) * N (digits [n][L][L+1][N], then [n][2][L+1][N]). */
he_status he_keyswitch_work_words(const he_ctx* ext, uint64_t n, uint64_t* words);

/* Client side (takes the secret key): the Galois key for g, written in NTT
 * form to d_ksk_ntt [L][2][L+1][N] as he_keyswitch and he_rotate read it:
 * k_a[l] = a[l], k_b[l] = a[l]*s + e[l] + G_l*s(X^g) over Z_QP.  d_sk: the
 * key's N integer coefficients (int64); d_a: [L][L+1][N] uniform residues
 * over q_0..q_{L-1}, P (canonical); d_err: int64 [L][N] small errors (random
 * values are the caller's).  d_work: (2L+2)*(L+1)*N words, clobbered.
 * g as for he_automorph; HE_EPARAM if ext->L < 2. */
he_status he_galois_key(const he_ctx* ext, uint64_t g, const int64_t* d_sk, const uint64_t* d_a, const int64_t* d_err,
                        uint64_t* d_ksk_ntt, uint64_t* d_work, void* stream);

/* The automorphism a(X) -> a(X^g) of n RNS polynomials [n][L][N] of `ctx`
 * (coefficient form, canonical): coefficient i moves to i*g mod 2N and is
 * negated when that index is N or more.  g odd with 0 < g < 2N, else
 * HE_EINVAL; out of place (d_in == d_out is HE_EINVAL).  Applied to both
 * components of a ciphertext it gives one of phase m(X^g) under s(X^g). */
he_status he_automorph(const he_ctx* ctx, uint64_t g, uint64_t n, const uint64_t* d_in, uint64_t* d_out,
                       void* stream);

/* Key switching of n ciphertexts from s' to s: digits d_l = limb l of a
 * (integers below q_l), A = sum_l d_l*k_a[l] and B = sum_l d_l*k_b[l] over
 * Z_QP, each divided by P with rounding (the residue mod P centred into
 * (-P/2, P/2]); d_out = (-A', b - B') mod Q, [n][2][L][N] canonical, written
 * completely; it may alias d_ct.  d_work: he_keyswitch_work_words words,
 * clobbered.  HE_EPARAM if ext->L < 2; HE_ESHAPE if n is too large for one
 * launch; n = 0 is a no-op. */
he_status he_keyswitch(const he_ctx* ext, uint64_t n, const uint64_t* d_ct, const uint64_t* d_ksk_ntt,
                       uint64_t* d_out, uint64_t* d_work, void* stream);

/* Rotation: he_automorph of both components by g, then he_keyswitch with a
 * key from s(X^g) to s; the automorphism is applied while the digits and b
 * are read, so the rotated ciphertext is never stored.  Out of place
 * (d_ct == d_out is HE_EINVAL); g as for he_automorph. */
he_status he_rotate(const he_ctx* ext, uint64_t g, uint64_t n, const uint64_t* d_ct, const uint64_t* d_ksk_ntt,
                    uint64_t* d_out, uint64_t* d_work, void* stream);

/* For callers that cannot allocate device memory or pass a work buffer
 * (code under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc): he_rotate with its key-switching scratch taken from a fixed
 * device array of the library instead of d_work.  The array holds
 * HE_ROTATE_NOALLOC_MAX_WORDS uint64 words (64 MiB) on every GPU the call
 * runs on, kept until the process ends; n is limited to what fits
 * (he_keyswitch_work_words(ext, n) <= that: 51 ciphertexts at N = 8192 with
 * 3 ciphertext primes), HE_ESHAPE beyond it.  No allocation and no library
 * routine that allocates.  Every call on one GPU shares that GPU's array:
 * calls that overlap on one GPU (several streams or host threads) race and
 * must be serialised by the caller.  Arguments and results otherwise as
 * he_rotate. */
#define HE_ROTATE_NOALLOC_MAX_WORDS (8ull * 1024 * 1024)
he_status he_rotate_noalloc(const he_ctx* ext, uint64_t g, uint64_t n, const uint64_t* d_ct,
                            const uint64_t* d_ksk_ntt, uint64_t* d_out, void* stream);

/* ------------------------------------------------------------------------
 * Z_P variant: batched plaintext slots over a prime t and the linear kernel
 * (Sec. 6.1: each iteration multiplies the input by NTT-preprocessed
 * weights, adds the product to the accumulated result and rotates it).
 * Slots: with t prime, t = 1 mod 2N, a plaintext m in Z_t[X]/(X^N+1) holds
 * in slot s = r*N/2 + j (row r < 2, column j < N/2) the value m(zeta^e),
 * e = 5^j mod 2N in row 0 and -5^j mod 2N in row 1, zeta = psi of t (the
 * transforms' root); X -> X^5 moves every row left by one slot.  Slot calls
 * take a T-CONTEXT: he_ctx_create with the single prime t (L = 1); other
 * contexts give HE_EPARAM.
 * ------------------------------------------------------------------------ */

/* Slots [n][N] (values in [0, t)) -> plaintext coefficients [n][N] as
 * integers centred into [-t/2, t/2) (int64), ready for he_encrypt (which
 * reduces them mod t) or he_zp_encode_plain.  d_slots != d_coeffs. */
he_status he_simd_encode(const he_ctx* tctx, uint64_t n, const uint64_t* d_slots, int64_t* d_coeffs, void* stream);

/* Plaintext coefficients [n][N] (any int64, e.g. he_decrypt's output) ->
 * slots [n][N] in [0, t).  d_work: [n][N] scratch. */
he_status he_simd_decode(const he_ctx* tctx, uint64_t n, const int64_t* d_coeffs, uint64_t* d_slots, uint64_t* d_work,
                         void* stream);

/* The n diagonals of the matrix W (int64 [rows][cols], row-major, rows,
 * cols <= n, zero-padded to n x n) as slot vectors [n][N] mod t: diagonal i
 * holds W[(k - i) mod n][k mod n] in slot k of each row.  n a power of two,
 * n <= N/2 (HE_ESHAPE otherwise).  With the input x repeated with period n
 * in the slots, sum_i rot^i(d_i * x) = W x in slots 0 .. rows-1. */
he_status he_zp_diagonals(const he_ctx* tctx, const int64_t* d_w, uint32_t rows, uint32_t cols, uint32_t n,
                          uint64_t* d_slots, void* stream);

/* The generalized diagonals of a matrix with fewer rows than columns:
 * n_out slot vectors [n_out][N], diagonal i holding W[(k - i) mod n_out][k mod
 * n_in] in slot k of each row (rows <= n_out <= n_in <= N/2, cols <= n_in,
 * powers of two; HE_ESHAPE otherwise).  With the input repeated with period
 * n_in, he_zp_matvec over these n_out diagonals leaves in slot
 * r + j*n_out the sum over columns r + j*n_out .. r + (j+1)*n_out - 1 of
 * row r; log2(n_in/n_out) he_zp_fold steps (rotations by n_out, 2*n_out,
 * ...) then give W x in slots 0 .. rows-1: n_out iterations instead of
 * n_in.  n_out = n_in is he_zp_diagonals. */
he_status he_zp_diagonals_rect(const he_ctx* tctx, const int64_t* d_w, uint32_t rows, uint32_t cols, uint32_t n_out,
                               uint32_t n_in, uint64_t* d_slots, void* stream);

/* Weight plaintexts for he_zp_matvec: coefficients [n][N] (centred int64,
 * from he_simd_encode) lifted to the L ciphertext primes of the EXTENDED
 * context (q_0..q_{L-1}, P), multiplied by -P mod q_l and transformed:
 * d_w [n][L][N] NTT form.  The factor -P lets the product enter key
 * switching's sums before the division by P. */
he_status he_zp_encode_plain(const he_ctx* ext, uint64_t n, const int64_t* d_coeffs, uint64_t* d_w, void* stream);

/* Words of scratch he_zp_matvec needs for n ciphertexts:
 * 2*n*2*L*N + n*(L+2)*(L+1)*N. */
he_status he_zp_work_words(const he_ctx* ext, uint64_t n, uint64_t* words);

/* The linear kernel on n input ciphertexts x (d_x_ntt: [n][2][L][N], NTT
 * form, e.g. he_ntt_fwd on the base context): acc = x * w_{D-1}; then for
 * i = D-2 down to 0, acc = rotate(acc, g) + x * w_i (D = n_diag, d_w from
 * he_zp_encode_plain, d_ksk_ntt the Galois key for g as for he_rotate).
 * Each iteration is one key switching whose inner product also takes the
 * plaintext term, so the product is never stored.  d_out: [n][2][L][N]
 * coefficient form (canonical).  With g = 5 and the diagonals of
 * he_zp_diagonals the slots of the result hold W x.  N <= 2^13 (HE_EPARAM
 * otherwise); d_work: he_zp_work_words words. */
he_status he_zp_matvec(const he_ctx* ext, uint64_t g, uint64_t n, const uint64_t* d_x_ntt, const uint64_t* d_w,
                       uint32_t n_diag, const uint64_t* d_ksk_ntt, uint64_t* d_out, uint64_t* d_work, void* stream);

/* One rotate-and-add step on n ciphertexts [n][2][L][N] (extended
 * context): d_out = d_ct + rotate(d_ct, g), with d_ksk_ntt the Galois key
 * for g as for he_rotate; the addition is folded into the last kernel.
 * Out of place (d_ct == d_out is HE_EINVAL); d_work: he_keyswitch_work_words
 * words. */
he_status he_zp_fold(const he_ctx* ext, uint64_t g, uint64_t n, const uint64_t* d_ct, const uint64_t* d_ksk_ntt,
                     uint64_t* d_out, uint64_t* d_work, void* stream);

/* Words of scratch he_zp_matvec_grouped needs: as he_zp_work_words for
 * groups*n ciphertexts. */
he_status he_zp_grouped_work_words(const he_ctx* ext, uint64_t n, uint32_t groups, uint64_t* words);

/* The same kernel scheduled as `groups` independent chains run as one
 * batch of groups*n ciphertexts: chain c takes the diagonals
 * c*per .. (c+1)*per - 1 (per = n_diag/groups) through the iteration above;
 * then acc = chain_{G-1} and acc = rotate(acc, g2) + chain_c for
 * c = G-2 .. 0, with g2 the Galois element of a rotation by per slots
 * (5^per mod 2N) and d_ksk2_ntt its key.  The same number of rotations in
 * per + groups - 1 dependent steps instead of n_diag, so a small batch
 * fills more of the GPU; the slots hold the same W x (the ciphertext words
 * differ from he_zp_matvec's).  n_diag % groups != 0 is HE_EINVAL; groups = 1
 * is he_zp_matvec. */
he_status he_zp_matvec_grouped(const he_ctx* ext, uint64_t g, uint64_t n, const uint64_t* d_x_ntt, const uint64_t* d_w,
                               uint32_t n_diag, uint32_t groups, const uint64_t* d_ksk_ntt, uint64_t g2,
                               const uint64_t* d_ksk2_ntt, uint64_t* d_out, uint64_t* d_work, void* stream);

/* ------------------------------------------------------------------------
 * Polyphase form of a strided convolution (a fusion variant of the layer:
 * the same outputs with fewer output ciphertexts when the packing keeps a
 * whole window per channel).  A stride-s conv (s >= 2) equals a stride-1,
 * pad-0 conv on s*s*C phase channels of the padded input, of size
 * ceil((H+2pad)/s) x ceil((W+2pad)/s), with a ceil(kh/s) x ceil(kw/s)
 * kernel; its first Ho x Wo outputs are the strided conv's (it may have a
 * few more rows or columns, which the caller ignores).  Phase channel
 * c*s*s + a*s + b holds xpad[c][s*y + a][s*x + b].  The layer itself runs
 * through the ordinary calls on the polyphase descriptor.
 * ------------------------------------------------------------------------ */

/* The polyphase descriptor of a strided conv (packing fields zero: plan it
 * with he_plan_conv).  HE_ESHAPE if stride < 2 or the shape is empty. */
he_status he_polyphase_desc(const he_conv_desc* in, he_conv_desc* out);

/* Host only: *use = 1 when the planner's objective (HBM bytes, then
 * modmuls; see he_plan_conv) is lower for the polyphase form of the strided
 * conv d at this batch than for the strided form, each with its own
 * planned packing; 0 otherwise, and for stride 1.  Packing fields of d are
 * ignored. */
he_status he_polyphase_advised(uint32_t N, uint32_t L, const he_conv_desc* d, uint32_t batch_hint, int* use);

/* Weights int64 [M][C][kh][kw] of the strided conv -> the polyphase conv's
 * [M][s*s*C][ceil(kh/s)][ceil(kw/s)]: Kp[m][c*s*s + a*s + b][i][j] =
 * K[m][c][s*i + a][s*j + b], zero outside the kernel (device buffers). */
he_status he_polyphase_weights(const he_conv_desc* desc, const int64_t* d_w, int64_t* d_wp, void* stream);

/* Inputs int64 [B][C][H][W] (e.g. the server's input share) -> the phase
 * channels [B][s*s*C][H'][W'], zero where the padded input is zero. */
he_status he_polyphase_input(const he_conv_desc* desc, uint32_t B, const int64_t* d_x, int64_t* d_xp, void* stream);

/* ------------------------------------------------------------------------
 * Batch executor: many layer solves of uneven shape in one launch.
 * Each job is one he_conv_layer call's worth of work (same buffers, same
 * result).  A batch runs the forward NTT of every job's input limb
 * polynomials as one grid, every job's MAC tiles as one grid and every
 * job's inverse NTTs as one grid (one workgroup per item), so small layers
 * no longer leave the GPU half empty.  With HE_SCHED_TWO_CHAINS the jobs are
 * split into two chains (balanced by weight bytes) on two streams, so the
 * MAC of one chain can overlap the transforms of the other.  With
 * use_graph the kernels of all chains are captured once into a hipGraph and
 * replayed with a single hipGraphLaunch.
 * ------------------------------------------------------------------------ */
typedef struct {
  he_conv_desc desc;      /* planned descriptor (Cw, Hw, Ww filled) */
  uint32_t B;             /* images in this job, >= 1 */
  uint64_t* d_in;         /* [B][CB][S][2][L][N] coefficient form; NTT'd in place (clobbered) */
  const uint64_t* d_wntt; /* [M][CB][L][N] from he_encode_weights */
  uint64_t* d_out;        /* [B][M][S][2][L][N] coefficient form, written completely */
} he_job;

typedef struct he_batch he_batch;

enum {
  HE_SCHED_ONE_CHAIN = 1,   /* one stream: all forward NTTs, all MACs, all inverse NTTs */
  HE_SCHED_TWO_CHAINS = 2,  /* two chains of jobs on two streams */
  HE_SCHED_PIPELINED_4 = 3, /* consecutive jobs in up to 4 groups of about equal MAC work: each
                               group's forward NTTs and MAC tiles on the caller's stream, its
                               inverse NTTs on a second stream once its MAC is done, beside the
                               next group's MAC */
  HE_SCHED_PIPELINED_8 = 4  /* the same in up to 8 groups */
};

/* Validate the jobs, build the work lists and copy them and the job table
 * to the device (the batch's only allocations, besides two streams and two
 * events for HE_SCHED_TWO_CHAINS).  The MAC register tile is the context's
 * (he_tuning mac_mt x mac_rt) when it is (4,4), (4,2), (2,4) or (2,2), else
 * (4,4), or (2,2) when a job has fewer than 4 ciphertext rows or output
 * channels.  The buffers named by the jobs must stay
 * allocated while the batch is used; jobs must not share input or output
 * buffers.  HE_EINVAL for an unknown schedule (value 0 named a persistent
 * single-kernel executor, which is disabled).  HE_ESHAPE for an invalid
 * descriptor or a grid larger than one launch covers (2^32 - 1 work-items:
 * 16,777,215 MAC tiles, 4,194,303 limb polynomials per transform grid). */
he_status he_batch_create(const he_ctx* ctx, const he_job* jobs, uint32_t n_jobs, uint32_t schedule,
                          he_batch** out);

/* Enqueue one execution of the whole batch on `stream` (use_graph = 0: the
 * kernels directly; else one hipGraphLaunch of the graph captured on first
 * use).  Executions of one batch must not overlap. */
he_status he_batch_launch(he_batch* b, void* stream, int use_graph);

/* One eager execution of the batch on `stream`, with HIP events around
 * each of its grids, for measurement: ms[3*c + p] receives the duration of
 * grid p (0 forward NTT, 1 MAC, 2 inverse NTT) of chain c, c < the chains
 * used (he_batch_info); an empty grid reads 0.  For the pipelined schedules
 * ms[0] and ms[1] are the sums of every group's forward-NTT and MAC grids
 * (caller's stream) and ms[5] the sum of the inverse-NTT grids (second
 * stream), each measured on its own; they overlap.  Same results as
 * he_batch_launch; synchronises `stream`.  Must not overlap another
 * execution of the batch. */
he_status he_batch_launch_timed(he_batch* b, void* stream, float* ms);

/* Synchronise `stream`; HE_EDEVICE if the device reported an error. */
he_status he_batch_status(he_batch* b, void* stream);

/* Work items over all grids, and streams used (1 or 2). */
he_status he_batch_info(const he_batch* b, uint64_t* n_items, uint32_t* n_chains);

/* The MAC form the batch picked (see he_tuning): the register tile
 * (mt, rt), the LDS stages (0: register loads), the tiles per workgroup of
 * the streamed MAC and whether its waves form the 2x2 grid.  Any output
 * pointer may be NULL. */
he_status he_batch_mac_form(const he_batch* b, uint32_t* mt, uint32_t* rt, uint32_t* lds, uint32_t* tiles,
                            uint32_t* grid);

void he_batch_destroy(he_batch* b);

#ifdef __cplusplus
}
#endif

#endif /* HECONV_H */
