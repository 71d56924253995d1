/*
 * CPU oracle for the homomorphic-convolution hot path (TEST INFRASTRUCTURE).
 *
 * This file is the slow, obviously correct reference that the HIP path is
 * checked against.  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may load it.  It shares no code, header, table or constant
 * generator with the product library.
 *
 * Arithmetic is exact: every product is formed in unsigned __int128 and
 * reduced with the C `%` operator.  Nothing is blocked, fused or reordered
 * beyond what the definitions below state.
 *
 * Paper passages followed (SecONNds, arXiv 2506.11586):
 *   - ring R_Q^N = Z_Q[X]/(X^N + 1)                        (Sec. 2.1)
 *   - RLWE/BFV encryption b = a*sk + delta*m + eps*e         (App. C)
 *   - polynomial product as a coefficient convolution        (App. C; the
 *     printed sum omits the negacyclic wrap term that X^N = -1 implies, and
 *     the wrap term is included here)
 *   - NTT-based multiplication: NTT both operands, Hadamard product, iNTT
 *                                                            (App. C.1)
 *   - NTT preprocessing: weights NTT'd once, ciphertexts NTT'd on receipt,
 *     every MAC in the NTT domain, only final results inverse-transformed
 *                                                            (Sec. 6.2)
 * The paper fixes no primes, no root of unity and no output order; the
 * readings used here (largest primes below 2^bits with q = 1 mod 2N, the
 * smallest primitive 2N-th root, bit-reversed evaluation order) are listed
 * with the design notes.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

static uint64_t mulmod(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)(((u128)a * b) % q); }
static uint64_t addmod(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)(((u128)a + b) % q); }
static uint64_t submod(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)(((u128)a + q - b) % q); }

static uint64_t powmod(uint64_t a, uint64_t e, uint64_t q) {
  uint64_t r = 1 % q;
  a %= q;
  while (e) {
    if (e & 1) r = mulmod(r, a, q);
    a = mulmod(a, a, q);
    e >>= 1;
  }
  return r;
}

/* Inverse by Fermat's little theorem (q prime). */
static uint64_t invmod(uint64_t a, uint64_t q) { return powmod(a, q - 2, q); }

/* ------------------------------------------------------------------------ */
/* Parameters                                                                */
/* ------------------------------------------------------------------------ */

/* Deterministic Miller-Rabin: the first twelve primes as bases decide every
 * n < 3.3e24, which covers all 64-bit n. */
int or_is_prime(uint64_t n) {
  static const uint64_t bases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  if (n < 2) return 0;
  for (int i = 0; i < 12; i++) {
    if (n == bases[i]) return 1;
    if (n % bases[i] == 0) return 0;
  }
  uint64_t d = n - 1;
  int s = 0;
  while ((d & 1) == 0) { d >>= 1; s++; }
  for (int i = 0; i < 12; i++) {
    uint64_t x = powmod(bases[i], d, n);
    if (x == 1 || x == n - 1) continue;
    int witness = 1;
    for (int r = 1; r < s; r++) {
      x = mulmod(x, x, n);
      if (x == n - 1) { witness = 0; break; }
    }
    if (witness) return 0;
  }
  return 1;
}

/* The L largest primes q < 2^bits with q = 1 (mod 2N), in descending order.
 * Returns the number found (L on success). */
int or_find_primes(uint32_t N, uint32_t bits, uint32_t L, uint64_t* out) {
  uint64_t step = 2ull * N;
  uint64_t top = (bits >= 64) ? ~0ull : ((1ull << bits) - 1);
  uint64_t q = (top - 1) / step * step + 1; /* largest value = 1 mod 2N not above top */
  uint32_t found = 0;
  while (found < L && q > step) {
    if (or_is_prime(q)) out[found++] = q;
    q -= step;
  }
  return (int)found;
}

/* Smallest primitive 2N-th root of unity mod q.  The primitive 2N-th roots
 * are exactly the N roots of x^N = -1 (2N is a power of two); given any one
 * of them, w, the full set is { w^k : k odd, k < 2N }, and the smallest
 * element of that set is returned.  w is found as x^((q-1)/2N) for the
 * first x >= 2 for which it satisfies w^N = -1. */
uint64_t or_find_psi(uint64_t q, uint32_t N) {
  uint64_t w = 0;
  for (uint64_t x = 2; x < q; x++) {
    uint64_t c = powmod(x, (q - 1) / (2ull * N), q);
    if (powmod(c, N, q) == q - 1) { w = c; break; }
  }
  if (w == 0) return 0;
  uint64_t best = w, w2 = mulmod(w, w, q), cur = w;
  for (uint32_t k = 1; k < 2 * N; k += 2) {
    if (cur < best) best = cur;
    cur = mulmod(cur, w2, q);
  }
  return best;
}

static uint32_t bitrev(uint32_t i, uint32_t logn) {
  uint32_t r = 0;
  for (uint32_t b = 0; b < logn; b++) r |= ((i >> b) & 1u) << (logn - 1 - b);
  return r;
}

static uint32_t ilog2(uint32_t n) {
  uint32_t l = 0;
  while ((1u << l) < n) l++;
  return l;
}

/* ------------------------------------------------------------------------ */
/* Ring products                                                             */
/* ------------------------------------------------------------------------ */

/* Schoolbook product in Z_q[X]/(X^N+1): c_k = sum_{i+j=k} a_i b_j
 * - sum_{i+j=k+N} a_i b_j.  O(N^2). */
void or_negacyclic_mul(const uint64_t* a, const uint64_t* b, uint64_t* c, uint32_t N, uint64_t q) {
  for (uint32_t k = 0; k < N; k++) c[k] = 0;
  for (uint32_t i = 0; i < N; i++) {
    if (a[i] == 0) continue;
    for (uint32_t j = 0; j < N; j++) {
      uint64_t p = mulmod(a[i], b[j], q);
      uint32_t k = i + j;
      if (k < N) c[k] = addmod(c[k], p, q);
      else c[k - N] = submod(c[k - N], p, q);
    }
  }
}

/* One coefficient k of the same product, O(N). */
uint64_t or_negacyclic_coeff(const uint64_t* a, const uint64_t* b, uint32_t k, uint32_t N, uint64_t q) {
  uint64_t acc = 0;
  for (uint32_t i = 0; i <= k; i++) acc = addmod(acc, mulmod(a[i], b[k - i], q), q);
  for (uint32_t i = k + 1; i < N; i++) acc = submod(acc, mulmod(a[i], b[N + k - i], q), q);
  return acc;
}

/* ------------------------------------------------------------------------ */
/* NTT by definition                                                         */
/* ------------------------------------------------------------------------ */

/* Forward negacyclic NTT by definition: out[i] = sum_j a[j] * psi^((2*brv(i)+1)*j),
 * i.e. the evaluation of a(X) at the odd powers of psi, listed in bit-reversed
 * order of the exponent.  O(N^2). */
void or_ntt_def(const uint64_t* a, uint64_t* out, uint32_t N, uint64_t q, uint64_t psi) {
  uint32_t logn = ilog2(N);
  for (uint32_t i = 0; i < N; i++) {
    uint64_t root = powmod(psi, 2ull * bitrev(i, logn) + 1, q);
    uint64_t acc = 0, pw = 1;
    for (uint32_t j = 0; j < N; j++) {
      acc = addmod(acc, mulmod(a[j], pw, q), q);
      pw = mulmod(pw, root, q);
    }
    out[i] = acc;
  }
}

/* Inverse by definition: out[j] = N^-1 * sum_i ahat[i] * psi^(-(2*brv(i)+1)*j). */
void or_intt_def(const uint64_t* ahat, uint64_t* out, uint32_t N, uint64_t q, uint64_t psi) {
  uint32_t logn = ilog2(N);
  uint64_t psi_inv = invmod(psi, q), n_inv = invmod(N % q, q);
  for (uint32_t j = 0; j < N; j++) out[j] = 0;
  for (uint32_t i = 0; i < N; i++) {
    uint64_t root = powmod(psi_inv, 2ull * bitrev(i, logn) + 1, q);
    uint64_t pw = 1;
    for (uint32_t j = 0; j < N; j++) {
      out[j] = addmod(out[j], mulmod(ahat[i], pw, q), q);
      pw = mulmod(pw, root, q);
    }
  }
  for (uint32_t j = 0; j < N; j++) out[j] = mulmod(out[j], n_inv, q);
}

/* ------------------------------------------------------------------------ */
/* NTT, textbook O(N log N) mode                                             */
/* ------------------------------------------------------------------------ */
/* The paper fixes the transform, not an algorithm for it.  This mode is the
 * textbook radix-2 split of X^N + 1 into (X^(N/2) - r)(X^(N/2) + r) with
 * r^2 = -1 repeated down to linear factors (Cooley-Tukey, natural order in,
 * bit-reversed order out), and its exact inverse (Gentleman-Sande).  It is
 * checked word for word against the definition above.
 * tab[k] = root^brv(k) (root = psi forward, psi^-1 inverse); every entry is an
 * independent powmod. */
static void twiddle_table(uint64_t* tab, uint32_t N, uint64_t q, uint64_t root) {
  uint32_t logn = ilog2(N);
  for (uint32_t k = 0; k < N; k++) tab[k] = powmod(root, bitrev(k, logn), q);
}

static void ntt_fast_tab(uint64_t* a, uint32_t N, uint64_t q, const uint64_t* tab) {
  uint32_t t = N;
  for (uint32_t m = 1; m < N; m <<= 1) {
    t >>= 1;
    for (uint32_t i = 0; i < m; i++) {
      uint64_t S = tab[m + i];
      uint32_t j1 = 2 * i * t;
      for (uint32_t j = j1; j < j1 + t; j++) {
        uint64_t U = a[j], V = mulmod(a[j + t], S, q);
        a[j] = addmod(U, V, q);
        a[j + t] = submod(U, V, q);
      }
    }
  }
}

static void intt_fast_tab(uint64_t* a, uint32_t N, uint64_t q, const uint64_t* itab) {
  uint64_t n_inv = invmod(N % q, q);
  uint32_t t = 1;
  for (uint32_t m = N; m > 1; m >>= 1) {
    uint32_t h = m >> 1, j1 = 0;
    for (uint32_t i = 0; i < h; i++) {
      uint64_t S = itab[h + i];
      for (uint32_t j = j1; j < j1 + t; j++) {
        uint64_t U = a[j], V = a[j + t];
        a[j] = addmod(U, V, q);
        a[j + t] = mulmod(submod(U, V, q), S, q);
      }
      j1 += 2 * t;
    }
    t <<= 1;
  }
  for (uint32_t j = 0; j < N; j++) a[j] = mulmod(a[j], n_inv, q);
}

void or_ntt_fast(uint64_t* a, uint32_t N, uint64_t q, uint64_t psi) {
  uint64_t* tab = (uint64_t*)malloc(sizeof(uint64_t) * N);
  twiddle_table(tab, N, q, psi);
  ntt_fast_tab(a, N, q, tab);
  free(tab);
}

void or_intt_fast(uint64_t* a, uint32_t N, uint64_t q, uint64_t psi) {
  uint64_t* tab = (uint64_t*)malloc(sizeof(uint64_t) * N);
  twiddle_table(tab, N, q, invmod(psi, q));
  intt_fast_tab(a, N, q, tab);
  free(tab);
}

/* Batched transforms over n RNS polynomials laid out [n][L][N]; limb l uses
 * q[l] and psi[l].  mode 0 = by definition, 1 = textbook fast mode. */
void or_ntt_batch(uint64_t* polys, uint64_t n, uint32_t L, uint32_t N, const uint64_t* q,
                  const uint64_t* psi, int mode, int inverse) {
  uint64_t* tabs = NULL;
  if (mode == 1) {
    tabs = (uint64_t*)malloc(sizeof(uint64_t) * N * L);
    for (uint32_t l = 0; l < L; l++)
      twiddle_table(tabs + (uint64_t)l * N, N, q[l], inverse ? invmod(psi[l], q[l]) : psi[l]);
  }
  long long total = (long long)(n * L);
#pragma omp parallel for schedule(dynamic)
  for (long long r = 0; r < total; r++) {
    uint32_t l = (uint32_t)(r % L);
    uint64_t* p = polys + (uint64_t)r * N;
    if (mode == 1) {
      if (inverse) intt_fast_tab(p, N, q[l], tabs + (uint64_t)l * N);
      else ntt_fast_tab(p, N, q[l], tabs + (uint64_t)l * N);
    } else {
      uint64_t* tmp = (uint64_t*)malloc(sizeof(uint64_t) * N);
      if (inverse) or_intt_def(p, tmp, N, q[l], psi[l]);
      else or_ntt_def(p, tmp, N, q[l], psi[l]);
      memcpy(p, tmp, sizeof(uint64_t) * N);
      free(tmp);
    }
  }
  free(tabs);
}

/* ------------------------------------------------------------------------ */
/* The convolution layer's arithmetic                                        */
/* ------------------------------------------------------------------------ */

/* Multiply-accumulate over channel blocks in the NTT domain (Sec. 6.2):
 *   out[b][m][s][c][l][k] = sum_{cb<CB} in[b][cb][s][c][l][k] * w[m][cb][l][k]  mod q_l
 * Layouts: in [B][CB][S][2][L][N], w [M][CB][L][N], out [B][M][S][2][L][N]. */
void or_conv_mac(const uint64_t* in, const uint64_t* w, uint64_t* out, uint32_t B, uint32_t CB, uint32_t S,
                 uint32_t M, uint32_t L, uint32_t N, const uint64_t* q) {
  long long rows = (long long)B * M * S * 2 * L;
#pragma omp parallel for schedule(static)
  for (long long r = 0; r < rows; r++) {
    long long x = r;
    uint32_t l = (uint32_t)(x % L); x /= L;
    uint32_t c = (uint32_t)(x % 2); x /= 2;
    uint32_t s = (uint32_t)(x % S); x /= S;
    uint32_t m = (uint32_t)(x % M); x /= M;
    uint32_t b = (uint32_t)x;
    uint64_t* o = out + (uint64_t)r * N;
    for (uint32_t k = 0; k < N; k++) {
      uint64_t acc = 0;
      for (uint32_t cb = 0; cb < CB; cb++) {
        const uint64_t* ip = in + ((((uint64_t)b * CB + cb) * S + s) * 2 + c) * L * N + (uint64_t)l * N;
        const uint64_t* wp = w + (((uint64_t)m * CB + cb) * L + l) * N;
        acc = addmod(acc, mulmod(ip[k], wp[k], q[l]), q[l]);
      }
      o[k] = acc;
    }
  }
}

/* The whole layer by its plain definition, in coefficient form:
 *   out[b][m][s][c][l] = sum_{cb} in[b][cb][s][c][l] (*) wc[m][cb][l]   in Z_{q_l}[X]/(X^N+1)
 * where (*) is the schoolbook negacyclic product and wc holds the packed weight
 * polynomials in coefficient form, layout [M][CB][L][N].  O(N^2) per product. */
void or_conv_layer_def(const uint64_t* in, const uint64_t* wc, uint64_t* out, uint32_t B, uint32_t CB, uint32_t S,
                       uint32_t M, uint32_t L, uint32_t N, const uint64_t* q) {
  long long rows = (long long)B * M * S * 2 * L;
#pragma omp parallel for schedule(dynamic)
  for (long long r = 0; r < rows; r++) {
    long long x = r;
    uint32_t l = (uint32_t)(x % L); x /= L;
    uint32_t c = (uint32_t)(x % 2); x /= 2;
    uint32_t s = (uint32_t)(x % S); x /= S;
    uint32_t m = (uint32_t)(x % M); x /= M;
    uint32_t b = (uint32_t)x;
    uint64_t* o = out + (uint64_t)r * N;
    uint64_t* prod = (uint64_t*)malloc(sizeof(uint64_t) * N);
    for (uint32_t k = 0; k < N; k++) o[k] = 0;
    for (uint32_t cb = 0; cb < CB; cb++) {
      const uint64_t* ip = in + ((((uint64_t)b * CB + cb) * S + s) * 2 + c) * L * N + (uint64_t)l * N;
      const uint64_t* wp = wc + (((uint64_t)m * CB + cb) * L + l) * N;
      or_negacyclic_mul(ip, wp, prod, N, q[l]);
      for (uint32_t k = 0; k < N; k++) o[k] = addmod(o[k], prod[k], q[l]);
    }
    free(prod);
  }
}

/* One output coefficient of the layer by definition, O(CB * N):
 * coefficient k of sum_cb in[b][cb][s][c][l] (*) wc[m][cb][l]. */
uint64_t or_conv_layer_coeff(const uint64_t* in, const uint64_t* wc, uint32_t CB, uint32_t S, uint32_t L, uint32_t N,
                             const uint64_t* q, uint32_t b, uint32_t m, uint32_t s, uint32_t c, uint32_t l,
                             uint32_t k) {
  uint64_t acc = 0;
  for (uint32_t cb = 0; cb < CB; cb++) {
    const uint64_t* ip = in + ((((uint64_t)b * CB + cb) * S + s) * 2 + c) * L * N + (uint64_t)l * N;
    const uint64_t* wp = wc + (((uint64_t)m * CB + cb) * L + l) * N;
    acc = addmod(acc, or_negacyclic_coeff(ip, wp, k, N, q[l]), q[l]);
  }
  return acc;
}

/* ------------------------------------------------------------------------ */
/* BFV client side (App. C), used only to make and open test ciphertexts      */
/* ------------------------------------------------------------------------ */

/* Negacyclic product of an arbitrary a (mod q) with a small signed s, by the
 * schoolbook sum (mode 0) or via the fast NTT (mode 1). */
static void mul_small(const uint64_t* a, const int64_t* s, uint64_t* out, uint32_t N, uint64_t q, uint64_t psi,
                      int mode) {
  uint64_t* sl = (uint64_t*)malloc(sizeof(uint64_t) * N);
  for (uint32_t i = 0; i < N; i++) sl[i] = s[i] >= 0 ? (uint64_t)s[i] % q : q - ((uint64_t)(-s[i]) % q);
  if (mode == 0) {
    or_negacyclic_mul(a, sl, out, N, q);
  } else {
    uint64_t* ah = (uint64_t*)malloc(sizeof(uint64_t) * N);
    memcpy(ah, a, sizeof(uint64_t) * N);
    or_ntt_fast(ah, N, q, psi);
    or_ntt_fast(sl, N, q, psi);
    for (uint32_t i = 0; i < N; i++) out[i] = mulmod(ah[i], sl[i], q);
    or_intt_fast(out, N, q, psi);
    free(ah);
  }
  free(sl);
}

/* Symmetric-key encryption of n messages.  Per message and limb:
 *   ct[0][l] = a_l,  ct[1][l] = a_l * sk + delta_l * m + e  (mod q_l)
 * a: [n][L][N] uniform words, e: [n][N] small signed, m: [n][N] in [0, t),
 * sk: [N] ternary; delta_l = floor(Q/t) mod q_l.  ct: [n][2][L][N]. */
void or_bfv_encrypt(uint64_t n, uint32_t L, uint32_t N, const uint64_t* q, const uint64_t* psi, const int64_t* sk,
                    const uint64_t* a, const int64_t* e, const uint64_t* m, const uint64_t* delta, uint64_t* ct,
                    int mode) {
  long long total = (long long)(n * L);
#pragma omp parallel for schedule(dynamic)
  for (long long r = 0; r < total; r++) {
    uint64_t i = (uint64_t)r / L;
    uint32_t l = (uint32_t)(r % L);
    const uint64_t* al = a + (i * L + l) * N;
    uint64_t* c0 = ct + ((i * 2 + 0) * L + l) * N;
    uint64_t* c1 = ct + ((i * 2 + 1) * L + l) * N;
    memcpy(c0, al, sizeof(uint64_t) * N);
    mul_small(al, sk, c1, N, q[l], psi[l], mode);
    for (uint32_t k = 0; k < N; k++) {
      int64_t ek = e[i * N + k];
      uint64_t el = ek >= 0 ? (uint64_t)ek % q[l] : q[l] - ((uint64_t)(-ek) % q[l]);
      c1[k] = addmod(addmod(c1[k], mulmod(delta[l], m[i * N + k] % q[l], q[l]), q[l]), el, q[l]);
    }
  }
}

/* Decryption phase per limb: v_l = ct[1][l] - ct[0][l] * sk (mod q_l).
 * ct: [n][2][L][N] -> v: [n][L][N].  CRT and rounding are done by the caller
 * in exact big-integer arithmetic. */
void or_bfv_phase(uint64_t n, uint32_t L, uint32_t N, const uint64_t* q, const uint64_t* psi, const int64_t* sk,
                  const uint64_t* ct, uint64_t* v, int mode) {
  long long total = (long long)(n * L);
#pragma omp parallel for schedule(dynamic)
  for (long long r = 0; r < total; r++) {
    uint64_t i = (uint64_t)r / L;
    uint32_t l = (uint32_t)(r % L);
    const uint64_t* c0 = ct + ((i * 2 + 0) * L + l) * N;
    const uint64_t* c1 = ct + ((i * 2 + 1) * L + l) * N;
    uint64_t* vl = v + (i * L + l) * N;
    mul_small(c0, sk, vl, N, q[l], psi[l], mode);
    for (uint32_t k = 0; k < N; k++) vl[k] = submod(c1[k], vl[k], q[l]);
  }
}

/* Number of OpenMP threads the parallel loops above use. */
int or_num_threads(void) {
  int n = 1;
#pragma omp parallel
  {
#pragma omp single
    {
#ifdef _OPENMP
      extern int omp_get_num_threads(void);
      n = omp_get_num_threads();
#endif
    }
  }
  return n;
}

/* Set the number of OpenMP threads of the parallel loops (n >= 1); used to
 * time the oracle on one core as well as on all of them. */
void or_set_threads(int n) {
#ifdef _OPENMP
  extern void omp_set_num_threads(int);
  omp_set_num_threads(n < 1 ? 1 : n);
#else
  (void)n;
#endif
}
