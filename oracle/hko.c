/*
 * Oracle (test infrastructure only) -- plain CPU reference for the fixed-point
 * LDL^T factorisation of the shifted Hankel moment matrix and the triangular
 * solves built on it.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library; the product path never
 * does.
 *
 * Arithmetic: the oracle's own sign-magnitude big integers with 32-bit digits
 * (schoolbook multiplication, Knuth's Algorithm D for division).  No external
 * bignum library and nothing shared with the GPU library.
 *
 * What it computes (paper, section "The LDL^T Determinant Algorithm"):
 *   - entries of M carry K fractional bits; the extracted column C and the
 *     quotients C/diag ("CDivDiag", called L here) carry K/2 = h fractional
 *     bits (the paragraph introducing the serial and parallel algorithms);
 *   - submatrix ("right-looking") order: column pc is extracted, divided by
 *     its diagonal entry and applied as a rank-1 update to every column to
 *     its right (serial algorithm, and the apply() routine of the parallel
 *     one);
 *   - the shift x is subtracted from the diagonal first (determinant()).
 * Rounding (the paper does not state one): round-to-nearest, ties-to-even,
 * at exactly two places -- C = RNE(A / 2^h) and L = RNE(C * 2^h / d) with
 * d = C[pc] the pivot actually used as divisor.  The rank-1 update itself is
 * exact (h + h = K fractional bits).
 *
 * Solves (not in the paper; needed by the inverse-iteration driver): see
 * hko_solve below for the fixed-point format and rounding points.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <stdio.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- bignum */
typedef struct {
  int neg;      /* 1 if negative (never set for zero) */
  int n;        /* number of significant digits (0 for zero) */
  int cap;
  uint32_t *d;  /* little-endian base-2^32 digits */
} bn;

static void bn_init(bn *a) { a->neg = 0; a->n = 0; a->cap = 0; a->d = NULL; }
static void bn_free(bn *a) { free(a->d); bn_init(a); }
static void bn_reserve(bn *a, int cap) {
  if (cap <= a->cap) return;
  int c = cap + 4;
  uint32_t *p = (uint32_t *)realloc(a->d, (size_t)c * sizeof(uint32_t));
  if (!p) { fprintf(stderr, "hko: out of memory\n"); abort(); }
  a->d = p; a->cap = c;
}
static void bn_trim(bn *a) {
  while (a->n > 0 && a->d[a->n - 1] == 0) a->n--;
  if (a->n == 0) a->neg = 0;
}
static void bn_copy(bn *r, const bn *a) {
  if (r == a) return;
  bn_reserve(r, a->n);
  if (a->n) memcpy(r->d, a->d, (size_t)a->n * sizeof(uint32_t));
  r->n = a->n; r->neg = a->neg;
}
static void bn_set_digits(bn *r, int neg, const uint32_t *d, int n) {
  bn_reserve(r, n);
  if (n) memcpy(r->d, d, (size_t)n * sizeof(uint32_t));
  r->n = n; r->neg = neg; bn_trim(r);
}
static long bn_bits(const bn *a) {
  if (a->n == 0) return 0;
  return 32L * (a->n - 1) + (32 - __builtin_clz(a->d[a->n - 1]));
}
static int mag_cmp(const uint32_t *a, int an, const uint32_t *b, int bnn) {
  if (an != bnn) return an < bnn ? -1 : 1;
  for (int i = an - 1; i >= 0; i--)
    if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1;
  return 0;
}
/* r = |a| + |b| (r may alias neither) */
static void mag_add(bn *r, const bn *a, const bn *b) {
  const bn *x = a->n >= b->n ? a : b, *y = a->n >= b->n ? b : a;
  bn_reserve(r, x->n + 1);
  uint64_t c = 0;
  int i = 0;
  for (; i < y->n; i++) { c += (uint64_t)x->d[i] + y->d[i]; r->d[i] = (uint32_t)c; c >>= 32; }
  for (; i < x->n; i++) { c += x->d[i]; r->d[i] = (uint32_t)c; c >>= 32; }
  r->d[i] = (uint32_t)c;
  r->n = x->n + 1;
}
/* r = |a| - |b|, requires |a| >= |b| (r may alias neither) */
static void mag_sub(bn *r, const bn *a, const bn *b) {
  bn_reserve(r, a->n);
  int64_t br = 0;
  int i = 0;
  for (; i < b->n; i++) {
    int64_t t = (int64_t)a->d[i] - b->d[i] - br;
    br = t < 0; r->d[i] = (uint32_t)(t + (br ? ((int64_t)1 << 32) : 0));
  }
  for (; i < a->n; i++) {
    int64_t t = (int64_t)a->d[i] - br;
    br = t < 0; r->d[i] = (uint32_t)(t + (br ? ((int64_t)1 << 32) : 0));
  }
  r->n = a->n;
}
/* r = a + (sign) b, signed; tmp must be distinct from everything */
static void bn_addsub(bn *r, const bn *a, const bn *b, int negate_b, bn *tmp) {
  int bneg = b->n ? (b->neg ^ negate_b) : 0;
  if (a->neg == bneg) {
    mag_add(tmp, a, b); tmp->neg = a->neg;
  } else if (mag_cmp(a->d, a->n, b->d, b->n) >= 0) {
    mag_sub(tmp, a, b); tmp->neg = a->neg;
  } else {
    mag_sub(tmp, b, a); tmp->neg = bneg;
  }
  bn_trim(tmp);
  bn_copy(r, tmp);
}
/* r = a * b (schoolbook); r distinct from a and b */
static void bn_mul(bn *r, const bn *a, const bn *b) {
  if (a->n == 0 || b->n == 0) { r->n = 0; r->neg = 0; return; }
  int n = a->n + b->n;
  bn_reserve(r, n);
  memset(r->d, 0, (size_t)n * sizeof(uint32_t));
  for (int i = 0; i < a->n; i++) {
    uint64_t c = 0, ai = a->d[i];
    uint32_t *rp = r->d + i;
    for (int j = 0; j < b->n; j++) {
      c += ai * b->d[j] + rp[j];
      rp[j] = (uint32_t)c; c >>= 32;
    }
    rp[b->n] = (uint32_t)c;
  }
  r->n = n; r->neg = a->neg ^ b->neg; bn_trim(r);
}
/* r = a * 2^s (s >= 0); r may alias a */
static void bn_shl(bn *r, const bn *a, long s) {
  if (a->n == 0) { r->n = 0; r->neg = 0; return; }
  int q = (int)(s / 32), b = (int)(s % 32), an = a->n, neg = a->neg;
  bn_reserve(r, an + q + 1);
  uint32_t top = 0;
  if (b) top = a->d[an - 1] >> (32 - b);
  for (int i = an - 1; i >= 0; i--) {
    uint32_t lo = (b && i > 0) ? (a->d[i - 1] >> (32 - b)) : 0;
    r->d[i + q] = b ? ((a->d[i] << b) | lo) : a->d[i];
  }
  for (int i = 0; i < q; i++) r->d[i] = 0;
  r->d[an + q] = top;
  r->n = an + q + 1; r->neg = neg; bn_trim(r);
}
/* r = floor(|a| / 2^s) as magnitude with a's sign; returns via out-params the
   bit just below the cut (half) and whether anything below it is nonzero. */
static void bn_shr_mag(bn *r, const bn *a, long s, int *half, int *sticky) {
  int q = (int)(s / 32), b = (int)(s % 32), an = a->n, neg = a->neg;
  *half = 0; *sticky = 0;
  if (s > 0) {
    long hb = s - 1;  /* bit index of the half bit */
    int hq = (int)(hb / 32), hbit = (int)(hb % 32);
    if (hq < an) *half = (a->d[hq] >> hbit) & 1;
    for (int i = 0; i < hq && i < an; i++) if (a->d[i]) { *sticky = 1; break; }
    if (!*sticky && hq < an && hbit > 0 && (a->d[hq] & ((1u << hbit) - 1))) *sticky = 1;
  }
  if (q >= an) { r->n = 0; r->neg = 0; return; }
  int rn = an - q;
  bn_reserve(r, rn);
  for (int i = 0; i < rn; i++) {
    uint32_t lo = a->d[i + q] >> b;
    uint32_t hi = (b && i + q + 1 < an) ? (a->d[i + q + 1] << (32 - b)) : 0;
    r->d[i] = b ? (lo | hi) : a->d[i + q];
  }
  r->n = rn; r->neg = neg; bn_trim(r);
}
/* add 1 to the magnitude */
static void mag_inc(bn *r) {
  bn_reserve(r, r->n + 1);
  for (int i = 0; i < r->n; i++) { if (++r->d[i] != 0) return; }
  r->d[r->n++] = 1;
}
/* r = RNE(a / 2^s), s >= 0; round-half-even is symmetric so it acts on the
   magnitude */
static void bn_rne_shr(bn *r, const bn *a, long s) {
  int neg = a->neg, half, sticky;
  if (s == 0) { bn_copy(r, a); return; }
  bn_shr_mag(r, a, s, &half, &sticky);
  int odd = r->n ? (r->d[0] & 1) : 0;
  if (half && (sticky || odd)) mag_inc(r);
  r->neg = r->n ? neg : 0;
}
/* Knuth, TAOCP vol. 2, 4.3.1, Algorithm D: q = floor(u/v), rem = u mod v on
   magnitudes.  v nonzero. */
static void mag_divmod(bn *q, bn *rem, const bn *u, const bn *v) {
  int n = v->n, m = u->n - v->n;
  if (mag_cmp(u->d, u->n, v->d, v->n) < 0) {
    q->n = 0; q->neg = 0; bn_copy(rem, u); rem->neg = 0; bn_trim(rem); return;
  }
  if (n == 1) {  /* short division */
    uint64_t rr = 0, dv = v->d[0];
    bn_reserve(q, u->n);
    for (int i = u->n - 1; i >= 0; i--) {
      uint64_t cur = (rr << 32) | u->d[i];
      q->d[i] = (uint32_t)(cur / dv); rr = cur % dv;
    }
    q->n = u->n; q->neg = 0; bn_trim(q);
    bn_reserve(rem, 1); rem->d[0] = (uint32_t)rr; rem->n = 1; rem->neg = 0; bn_trim(rem);
    return;
  }
  int s = __builtin_clz(v->d[n - 1]);
  uint32_t *vn = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
  uint32_t *un = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(u->n + 1));
  for (int i = n - 1; i > 0; i--)
    vn[i] = s ? (v->d[i] << s) | (v->d[i - 1] >> (32 - s)) : v->d[i];
  vn[0] = v->d[0] << s;
  un[u->n] = s ? (u->d[u->n - 1] >> (32 - s)) : 0;
  for (int i = u->n - 1; i > 0; i--)
    un[i] = s ? (u->d[i] << s) | (u->d[i - 1] >> (32 - s)) : u->d[i];
  un[0] = u->d[0] << s;
  bn_reserve(q, m + 1);
  const uint64_t B = (uint64_t)1 << 32;
  for (int j = m; j >= 0; j--) {
    uint64_t num = ((uint64_t)un[j + n] << 32) | un[j + n - 1];
    uint64_t qhat = num / vn[n - 1], rhat = num % vn[n - 1];
    while (qhat >= B || qhat * vn[n - 2] > ((rhat << 32) | un[j + n - 2])) {
      qhat--; rhat += vn[n - 1];
      if (rhat >= B) break;
    }
    /* un[j..j+n] -= qhat * vn */
    int64_t borrow = 0;
    uint64_t carry = 0;
    for (int i = 0; i < n; i++) {
      uint64_t p = qhat * vn[i] + carry;
      carry = p >> 32;
      int64_t t = (int64_t)un[i + j] - (int64_t)(p & 0xffffffffu) - borrow;
      un[i + j] = (uint32_t)t;
      borrow = t < 0 ? 1 : 0;
    }
    int64_t t = (int64_t)un[j + n] - (int64_t)carry - borrow;
    un[j + n] = (uint32_t)t;
    if (t < 0) {  /* qhat was one too large: add v back */
      qhat--;
      uint64_t c = 0;
      for (int i = 0; i < n; i++) {
        c += (uint64_t)un[i + j] + vn[i];
        un[i + j] = (uint32_t)c; c >>= 32;
      }
      un[j + n] = (uint32_t)(un[j + n] + c);
    }
    q->d[j] = (uint32_t)qhat;
  }
  q->n = m + 1; q->neg = 0; bn_trim(q);
  bn_reserve(rem, n);
  for (int i = 0; i < n; i++)
    rem->d[i] = s ? (un[i] >> s) | (un[i + 1] << (32 - s)) : un[i];
  rem->n = n; rem->neg = 0; bn_trim(rem);
  free(vn); free(un);
}
/* r = RNE(a / b), b != 0, signed. */
static void bn_rne_div(bn *r, const bn *a, const bn *b, bn *t1, bn *t2) {
  int neg = a->neg ^ b->neg;
  bn ua = *a, ub = *b; ua.neg = 0; ub.neg = 0;   /* shallow views */
  mag_divmod(r, t1, &ua, &ub);
  /* compare 2*rem with |b| */
  bn_shl(t2, t1, 1);
  int c = mag_cmp(t2->d, t2->n, b->d, b->n);
  int odd = r->n ? (r->d[0] & 1) : 0;
  if (c > 0 || (c == 0 && odd)) mag_inc(r);
  r->neg = r->n ? neg : 0;
}

/* ------------------------------------------------------- interchange I/O */
/* A list of big integers crosses the boundary as (slen[i], off[i], digits):
   |slen| = number of 32-bit digits, sign of slen = sign of the value. */
static void bn_from_io(bn *r, int32_t slen, const uint32_t *dig) {
  int n = slen < 0 ? -slen : slen;
  bn_set_digits(r, slen < 0, dig, n);
}

/* ------------------------------------------------------ factorisation */
typedef struct {
  int N, K, h;
  bn *C;        /* column pc: entries r = pc..N-1 at C[cidx(pc, r)] */
  bn *L;        /* column pc: entries r = pc+1..N-1 at L[lidx(pc, r)] */
  int first_nonpos;   /* first pivot index with d <= 0 (-1 if none) */
  int nneg;           /* number of negative pivots */
  int status;         /* 0 ok, 1 zero pivot met (factorisation stopped) */
  double limb_macs;   /* sum over updates of ndig(C) * ndig(L) */
} hko_fact;

static inline size_t tri_idx(int N, int c, int r) {  /* r >= c */
  return (size_t)c * N - (size_t)c * (c - 1) / 2 + (size_t)(r - c);
}
static inline size_t lidx(int N, int c, int r) {     /* r > c, strictly lower */
  return (size_t)c * (N - 1) - (size_t)c * (c - 1) / 2 + (size_t)(r - c - 1);
}

void hko_fact_free(hko_fact *f) {
  if (!f) return;
  size_t nc = (size_t)f->N * (f->N + 1) / 2, nl = (size_t)f->N * (f->N - 1) / 2;
  for (size_t i = 0; i < nc; i++) bn_free(&f->C[i]);
  for (size_t i = 0; i < nl; i++) bn_free(&f->L[i]);
  free(f->C); free(f->L); free(f);
}

/* Factor M - x I where M_rc = X[r + c] / 2^K (X: 2N-1 integers) and the
   shift x = xs / 2^K.  Stops after the first `ncols` columns when
   0 < ncols < N (prefix factorisation, used for sampled checks). */
hko_fact *hko_factor(int N, int K, const int32_t *xslen, const int64_t *xoff,
                     const uint32_t *xdig, int32_t shift_slen,
                     const uint32_t *shift_dig, int ncols, int nthreads) {
  if (N < 1 || K < 2 || (K & 1)) return NULL;
  if (ncols <= 0 || ncols > N) ncols = N;
  int h = K / 2;
  hko_fact *f = (hko_fact *)calloc(1, sizeof(hko_fact));
  f->N = N; f->K = K; f->h = h; f->first_nonpos = -1;
  size_t ntri = (size_t)N * (N + 1) / 2, nl = (size_t)N * (N - 1) / 2;
  f->C = (bn *)calloc(ntri, sizeof(bn));
  f->L = (bn *)calloc(nl ? nl : 1, sizeof(bn));
  bn *A = (bn *)calloc(ntri, sizeof(bn));
  bn *X = (bn *)calloc((size_t)2 * N - 1, sizeof(bn));
  for (int i = 0; i < 2 * N - 1; i++) bn_from_io(&X[i], xslen[i], xdig + xoff[i]);
  bn xs; bn_init(&xs); bn_from_io(&xs, shift_slen, shift_dig);
  bn t1, t2; bn_init(&t1); bn_init(&t2);
  /* A = M - xI (lower triangle), determinant(): diagonal shift first */
  for (int c = 0; c < N; c++)
    for (int r = c; r < N; r++) {
      bn *a = &A[tri_idx(N, c, r)];
      bn_copy(a, &X[r + c]);
      if (r == c) bn_addsub(a, a, &xs, 1, &t1);
    }
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
  double macs = 0.0;
  for (int pc = 0; pc < ncols; pc++) {
    /* extract the column with h fractional bits */
    for (int r = pc; r < N; r++) bn_rne_shr(&f->C[tri_idx(N, pc, r)], &A[tri_idx(N, pc, r)], h);
    bn *d = &f->C[tri_idx(N, pc, pc)];
    if (d->n == 0 || d->neg) {
      if (f->first_nonpos < 0) f->first_nonpos = pc;
      if (d->neg) f->nneg++;
    }
    if (pc == N - 1) break;
    if (d->n == 0) { f->status = 1; break; }
    /* L = C * 2^h / d, exactly rounded */
#pragma omp parallel
    {
      bn u, a1, a2; bn_init(&u); bn_init(&a1); bn_init(&a2);
#pragma omp for schedule(dynamic, 8)
      for (int r = pc + 1; r < N; r++) {
        bn_shl(&u, &f->C[tri_idx(N, pc, r)], h);
        bn_rne_div(&f->L[lidx(N, pc, r)], &u, d, &a1, &a2);
      }
      bn_free(&u); bn_free(&a1); bn_free(&a2);
    }
    /* rank-1 update of the trailing triangle (exact) */
#pragma omp parallel reduction(+ : macs)
    {
      bn p, tmp; bn_init(&p); bn_init(&tmp);
#pragma omp for schedule(dynamic, 1)
      for (int c = pc + 1; c < N; c++) {
        const bn *cc = &f->C[tri_idx(N, pc, c)];
        for (int r = c; r < N; r++) {
          const bn *ll = &f->L[lidx(N, pc, r)];
          macs += (double)cc->n * (double)ll->n;
          bn_mul(&p, cc, ll);
          bn *a = &A[tri_idx(N, c, r)];
          bn_addsub(a, a, &p, 1, &tmp);
        }
      }
      bn_free(&p); bn_free(&tmp);
    }
  }
  f->limb_macs = macs;
  for (size_t i = 0; i < ntri; i++) bn_free(&A[i]);
  for (int i = 0; i < 2 * N - 1; i++) bn_free(&X[i]);
  free(A); free(X);
  bn_free(&xs); bn_free(&t1); bn_free(&t2);
  return f;
}

int hko_fact_info(const hko_fact *f, int *first_nonpos, int *nneg, double *limb_macs) {
  *first_nonpos = f->first_nonpos; *nneg = f->nneg; *limb_macs = f->limb_macs;
  return f->status;
}

/* Export: kind 0 = C (column pc, rows pc..N-1), kind 1 = L (column pc, rows
   pc+1..N-1), kind 2 = pivots d_pc = C_pc[pc].  Columns [c0, c1).  First call
   with dig == NULL returns the number of digits needed. */
static const bn *fact_item(const hko_fact *f, int kind, int pc, int r) {
  if (kind == 1) return &f->L[lidx(f->N, pc, r)];
  return &f->C[tri_idx(f->N, pc, r)];
}
int64_t hko_fact_export(const hko_fact *f, int kind, int c0, int c1,
                        int32_t *slen, int64_t *off, uint32_t *dig) {
  int64_t pos = 0, k = 0;
  for (int pc = c0; pc < c1; pc++) {
    int rlo = kind == 0 ? pc : (kind == 1 ? pc + 1 : pc), rhi = kind == 2 ? pc + 1 : f->N;
    for (int r = rlo; r < rhi; r++) {
      const bn *a = fact_item(f, kind, pc, r);
      if (dig) {
        slen[k] = a->neg ? -a->n : a->n;
        off[k] = pos;
        if (a->n) memcpy(dig + pos, a->d, (size_t)a->n * sizeof(uint32_t));
      }
      pos += a->n; k++;
    }
  }
  return pos;
}

/* -------------------------------------------------------------- vectors */
typedef struct { int n; bn *v; } hko_vec;

hko_vec *hko_vec_new(int n, const int32_t *slen, const int64_t *off, const uint32_t *dig) {
  hko_vec *v = (hko_vec *)calloc(1, sizeof(hko_vec));
  v->n = n; v->v = (bn *)calloc((size_t)(n ? n : 1), sizeof(bn));
  for (int i = 0; i < n && slen; i++) bn_from_io(&v->v[i], slen[i], dig + off[i]);
  return v;
}
void hko_vec_free(hko_vec *v) {
  if (!v) return;
  for (int i = 0; i < v->n; i++) bn_free(&v->v[i]);
  free(v->v); free(v);
}
int64_t hko_vec_export(const hko_vec *v, int32_t *slen, int64_t *off, uint32_t *dig) {
  int64_t pos = 0;
  for (int i = 0; i < v->n; i++) {
    const bn *a = &v->v[i];
    if (dig) {
      slen[i] = a->neg ? -a->n : a->n; off[i] = pos;
      if (a->n) memcpy(dig + pos, a->d, (size_t)a->n * sizeof(uint32_t));
    }
    pos += a->n;
  }
  return pos;
}

/* y = (L D L^T)^{-1} b.  b carries K fractional bits; z, w and y carry
   F = K + g fractional bits (g >= 0 guard bits, a reading: fixed-point
   rounding of z and w is amplified by the large entries of L^{-T}, so the
   intermediate vectors keep g extra bits).  Every inner product is exact and
   rounded once:
     z_i = RNE((b_i 2^(h+g) - sum_{k<i} L_k[i] z_k) / 2^h)
     w_i = RNE(z_i 2^h / d_i)
     y_i = RNE((w_i 2^h - sum_{k>i} L_i[k] y_k) / 2^h)
   stage: 1 = forward only (z), 2 = forward + diagonal (w), 3 = full (y). */
hko_vec *hko_solve(const hko_fact *f, const hko_vec *b, int stage, int g) {
  int N = f->N, h = f->h;
  if (b->n != N || f->status != 0 || g < 0) return NULL;
  hko_vec *y = hko_vec_new(N, NULL, NULL, NULL);
  bn acc, p, tmp, t1, t2; bn_init(&acc); bn_init(&p); bn_init(&tmp); bn_init(&t1); bn_init(&t2);
  /* forward: L z = b, L unit lower triangular with L[i][k] = L_k[i] */
  for (int i = 0; i < N; i++) {
    bn_shl(&acc, &b->v[i], h + g);
    for (int k = 0; k < i; k++) {
      bn_mul(&p, &f->L[lidx(N, k, i)], &y->v[k]);
      bn_addsub(&acc, &acc, &p, 1, &tmp);
    }
    bn_rne_shr(&y->v[i], &acc, h);
  }
  if (stage >= 2) {  /* w_i = RNE(z_i 2^h / d_i) */
    for (int i = 0; i < N; i++) {
      const bn *d = &f->C[tri_idx(N, i, i)];
      if (d->n == 0) { hko_vec_free(y); y = NULL; goto out; }
      bn_shl(&acc, &y->v[i], h);
      bn_rne_div(&y->v[i], &acc, d, &t1, &t2);
    }
  }
  if (stage >= 3) {  /* backward: L^T y = w */
    for (int i = N - 1; i >= 0; i--) {
      bn_shl(&acc, &y->v[i], h);
      for (int k = i + 1; k < N; k++) {
        bn_mul(&p, &f->L[lidx(N, i, k)], &y->v[k]);
        bn_addsub(&acc, &acc, &p, 1, &tmp);
      }
      bn_rne_shr(&y->v[i], &acc, h);
    }
  }
out:
  bn_free(&acc); bn_free(&p); bn_free(&tmp); bn_free(&t1); bn_free(&t2);
  return y;
}

/* ------------------------------------------- primitive checks (for pins) */
/* Expose the digit-level primitives so that tests can pin them against an
   independent big-integer implementation.  op: 0 mul, 1 add, 2 sub,
   3 RNE(a / 2^s), 4 RNE(a / b), 5 a * 2^s, 6 floor(|a|/|b|), 7 |a| mod |b| */
int64_t hko_prim(int op, int32_t aslen, const uint32_t *ad, int32_t bslen,
                 const uint32_t *bd, long s, int32_t *rslen, uint32_t *rd, int64_t cap) {
  bn a, b, r, t1, t2; bn_init(&a); bn_init(&b); bn_init(&r); bn_init(&t1); bn_init(&t2);
  bn_from_io(&a, aslen, ad); bn_from_io(&b, bslen, bd);
  switch (op) {
    case 0: bn_mul(&r, &a, &b); break;
    case 1: bn_addsub(&r, &a, &b, 0, &t1); break;
    case 2: bn_addsub(&r, &a, &b, 1, &t1); break;
    case 3: bn_rne_shr(&r, &a, s); break;
    case 4: bn_rne_div(&r, &a, &b, &t1, &t2); break;
    case 5: bn_shl(&r, &a, s); break;
    case 6: { bn ua = a, ub = b; ua.neg = 0; ub.neg = 0; mag_divmod(&r, &t1, &ua, &ub); } break;
    case 7: { bn ua = a, ub = b; ua.neg = 0; ub.neg = 0; mag_divmod(&t1, &r, &ua, &ub); } break;
    default: break;
  }
  int64_t n = r.n;
  if (n <= cap) { *rslen = r.neg ? -r.n : r.n; if (n) memcpy(rd, r.d, (size_t)n * 4); }
  bn_free(&a); bn_free(&b); bn_free(&r); bn_free(&t1); bn_free(&t2);
  (void)bn_bits;
  return n;
}

int hko_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
