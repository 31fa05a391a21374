/*
 * synth.c -- seeded synthetic genotype inputs in the packed 2-bit layout.
 *
 * This module only draws random genotypes and packs them. It contains no part
 * of the correlation method (no decoding, tallying or formula): both the CPU
 * oracle and the GPU library consume what it writes, and neither links it.
 *
 * Packed layout (one row per vector, `ld` bytes per row, ld % 16 == 0):
 *   field q of vector i sits in byte i*ld + q/4, bits 2*(q%4) (low) and
 *   2*(q%4)+1 (high).  The 2-bit code is the allele pair itself, high bit
 *   first: 0b00 = (0,0), 0b01 = (0,1), 0b11 = (1,1); 0b10 = (1,0) is the
 *   marker for a missing entry (the paper's future-work section reserves it).
 *   Bits past n_f in a row are padding.
 *
 * Random numbers come from a counter-based generator: the SplitMix64 output
 * function (Steele, Lea and Flood, OOPSLA 2014) applied to a key built from
 * (seed, stream tag, vector index, field index), so every entry is a pure
 * function of its coordinates and any sub-range can be regenerated alone.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define CODE_00 0u
#define CODE_01 1u
#define CODE_MISSING 2u
#define CODE_11 3u

static inline uint64_t sm64_mix(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* Key for coordinate (tag, a, b) under `seed`. */
static inline uint64_t ctr_hash(uint64_t seed, uint64_t tag, uint64_t a, uint64_t b) {
  uint64_t h = sm64_mix(seed ^ (tag * 0xD1B54A32D192ED03ull));
  h = sm64_mix(h ^ a);
  return sm64_mix(h ^ (b * 0xA0761D6478BD642Full));
}

/* Uniform double in [0,1) from the top 53 bits. */
static inline double u53(uint64_t h) { return (double)(h >> 11) * (1.0 / 9007199254740992.0); }
/* Uniform double in [0,1) from the low 32 bits (independent of u53's bits). */
static inline double u32lo(uint64_t h) { return (double)(h & 0xFFFFFFFFull) * (1.0 / 4294967296.0); }

enum { TAG_P = 1, TAG_G = 2, TAG_PAD = 3, TAG_SIZE = 4, TAG_W = 5, TAG_MP = 6, TAG_MG = 7,
       TAG_MG2 = 8 };

static inline void put_code(uint8_t* row, int64_t q, unsigned code) {
  uint8_t* b = row + (q >> 2);
  int sh = (int)(q & 3) * 2;
  *b = (uint8_t)((*b & ~(3u << sh)) | ((code & 3u) << sh));
}

/* Fill bits past n_f: pad_mode 0 = zero bits, 1 = random garbage. */
static void fill_padding(uint8_t* row, int64_t n_f, int64_t ld, uint64_t seed, int64_t i,
                         int pad_mode) {
  int64_t total = ld * 4;
  for (int64_t q = n_f; q < total; ++q) {
    unsigned c = 0;
    if (pad_mode == 1) c = (unsigned)(ctr_hash(seed, TAG_PAD, (uint64_t)i, (uint64_t)q) & 3u);
    put_code(row, q, c);
  }
}

/*
 * Genotypes uniform over {00, 01, 11}, then each entry replaced by the
 * missing code with probability `missing`.
 */
void synth_uniform(uint8_t* v, int64_t n_v, int64_t n_f, int64_t ld, uint64_t seed,
                   double missing, int pad_mode) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n_v; ++i) {
    uint8_t* row = v + i * ld;
    memset(row, 0, (size_t)ld);
    for (int64_t q = 0; q < n_f; ++q) {
      uint64_t h = ctr_hash(seed, TAG_G, (uint64_t)i, (uint64_t)q);
      double u = u53(h);
      unsigned g = u < (1.0 / 3.0) ? CODE_00 : (u < (2.0 / 3.0) ? CODE_01 : CODE_11);
      if (missing > 0.0 && u32lo(h) < missing) g = CODE_MISSING;
      put_code(row, q, g);
    }
    fill_padding(row, n_f, ld, seed, i, pad_mode);
  }
}

/* Per-vector allele-0 frequency p_i ~ Beta(1/2, 1/2) (the arcsine law):
 * p = sin^2(pi u / 2) with u uniform. */
double synth_beta_half(uint64_t seed, int64_t i) {
  double u = u53(ctr_hash(seed, TAG_P, (uint64_t)i, 0));
  double s = sin(1.5707963267948966 * u);
  return s * s;
}

/*
 * Hardy-Weinberg genotypes: P(00) = p^2, P(01) = 2p(1-p), P(11) = (1-p)^2
 * with p = p_i ~ Beta(1/2,1/2) per vector; then missing with probability
 * `missing`, independently per entry.
 */
void synth_beta_hw(uint8_t* v, int64_t n_v, int64_t n_f, int64_t ld, uint64_t seed,
                   double missing, int pad_mode) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n_v; ++i) {
    uint8_t* row = v + i * ld;
    memset(row, 0, (size_t)ld);
    double p = synth_beta_half(seed, i);
    double t0 = p * p;
    double t1 = t0 + 2.0 * p * (1.0 - p);
    /* Build whole bytes to keep the generator fast on large inputs. */
    for (int64_t q0 = 0; q0 < n_f; q0 += 4) {
      unsigned byte = 0;
      for (int t = 0; t < 4 && q0 + t < n_f; ++t) {
        uint64_t h = ctr_hash(seed, TAG_G, (uint64_t)i, (uint64_t)(q0 + t));
        double u = u53(h);
        unsigned g = u < t0 ? CODE_00 : (u < t1 ? CODE_01 : CODE_11);
        if (missing > 0.0 && u32lo(h) < missing) g = CODE_MISSING;
        byte |= g << (2 * t);
      }
      row[q0 >> 2] = (uint8_t)byte;
    }
    fill_padding(row, n_f, ld, seed, i, pad_mode);
  }
}

/*
 * Analytically checkable placement input: vector i holds 11 on fields
 * q = 0 mod s[i] and 00 elsewhere (no missing entries).
 */
void synth_placement(uint8_t* v, int64_t n_v, int64_t n_f, int64_t ld, const int64_t* s,
                     uint64_t seed, int pad_mode) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n_v; ++i) {
    uint8_t* row = v + i * ld;
    memset(row, 0, (size_t)ld);
    for (int64_t q = 0; q < n_f; ++q) put_code(row, q, (q % s[i]) == 0 ? CODE_11 : CODE_00);
    fill_padding(row, n_f, ld, seed, i, pad_mode);
  }
}

/* Constant code everywhere (used for closed-form cases). */
void synth_constant(uint8_t* v, int64_t n_v, int64_t n_f, int64_t ld, const uint8_t* codes,
                    uint64_t seed, int pad_mode) {
  for (int64_t i = 0; i < n_v; ++i) {
    uint8_t* row = v + i * ld;
    memset(row, 0, (size_t)ld);
    for (int64_t q = 0; q < n_f; ++q) put_code(row, q, codes[i]);
    fill_padding(row, n_f, ld, seed, i, pad_mode);
  }
}

/*
 * Sizes for a batch of independent problems: n_v = floor(exp(U(ln lo, ln hi)))
 * and n_f uniform on the integers [f_lo, f_hi].
 */
void synth_batch_sizes(int64_t n_probs, uint64_t seed, int64_t v_lo, int64_t v_hi, int64_t f_lo,
                       int64_t f_hi, int64_t* n_v_out, int64_t* n_f_out) {
  double a = log((double)v_lo), b = log((double)v_hi);
  for (int64_t p = 0; p < n_probs; ++p) {
    double u = u53(ctr_hash(seed, TAG_SIZE, (uint64_t)p, 0));
    int64_t nv = (int64_t)floor(exp(a + (b - a) * u));
    if (nv < v_lo) nv = v_lo;
    if (nv > v_hi) nv = v_hi;
    n_v_out[p] = nv;
    uint64_t h = ctr_hash(seed, TAG_SIZE, (uint64_t)p, 1);
    n_f_out[p] = f_lo + (int64_t)(h % (uint64_t)(f_hi - f_lo + 1));
  }
}

/* Random weights in [0, 2^61 - 1) for whole-output checksums. */
void synth_weights(uint64_t* w, int64_t n, uint64_t seed, uint64_t tag) {
  const uint64_t P61 = (1ull << 61) - 1;
  for (int64_t i = 0; i < n; ++i) w[i] = ctr_hash(seed, TAG_W + tag, (uint64_t)i, 7) % P61;
}

/*
 * Multi-allelic genotypes in the one-byte count layout: one byte per field,
 * `ld` bytes per row; bits 2a and 2a+1 of the byte hold how many of the
 * entry's two alleles are state a (a < s <= 4), and a missing entry is the
 * byte 0.  Per vector, state weights sin^2(pi u_a / 2) (u_a uniform) are
 * normalised into allele frequencies; the two alleles of an entry are
 * independent draws from them (Hardy-Weinberg); then the entry is replaced by
 * the missing byte with probability `missing`.  Bytes past n_f are padding
 * (zero, or random garbage with pad_mode 1).
 */
void synth_multi_hw(uint8_t* v, int64_t n_v, int64_t n_f, int64_t ld, int s, uint64_t seed,
                    double missing, int pad_mode) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n_v; ++i) {
    uint8_t* row = v + i * ld;
    double cdf[4] = {0.0, 0.0, 0.0, 0.0}, tot = 0.0;
    for (int a = 0; a < s; ++a) {
      double sn = sin(1.5707963267948966 * u53(ctr_hash(seed, TAG_MP, (uint64_t)i, (uint64_t)a)));
      tot += sn * sn + 1e-3;
      cdf[a] = tot;
    }
    for (int64_t q = 0; q < n_f; ++q) {
      uint64_t h1 = ctr_hash(seed, TAG_MG, (uint64_t)i, (uint64_t)q);
      uint64_t h2 = ctr_hash(seed, TAG_MG2, (uint64_t)i, (uint64_t)q);
      double x1 = u53(h1) * tot, x2 = u53(h2) * tot;
      int a1 = 0, a2 = 0;
      while (a1 < s - 1 && x1 >= cdf[a1]) ++a1;
      while (a2 < s - 1 && x2 >= cdf[a2]) ++a2;
      unsigned byte = (1u << (2 * a1)) + (1u << (2 * a2));
      if (missing > 0.0 && u32lo(h2) < missing) byte = 0u;
      row[q] = (uint8_t)byte;
    }
    for (int64_t q = n_f; q < ld; ++q)
      row[q] = pad_mode == 1 ? (uint8_t)ctr_hash(seed, TAG_PAD, (uint64_t)i, (uint64_t)q) : 0;
  }
}
