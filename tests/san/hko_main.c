/* CPU harness for the sanitizer build of the oracle (test infrastructure).
   Compiled together with the oracle's own source under AddressSanitizer and
   UndefinedBehaviorSanitizer; reads a job from stdin and prints results in
   hexadecimal so that the test compares them with the ordinary build.

   Job "factor":  N K g, then 2N-1 moments, the shift, N right-hand-side
                  entries (one signed hexadecimal integer per line).  Prints
                  "C pc r v" and "L pc r v" for every entry, then "Y i v" for
                  the full solve with guard g.
   Job "prim":    lines "op s a b" until end of input; prints one result per
                  line (op codes as in hko_prim). */
#include "../../oracle/hko.c"

#include <stdio.h>

static char line[1 << 20];

static int read_hex(bn *r) {
  if (!fgets(line, sizeof line, stdin)) return 0;
  char *p = line;
  int neg = 0;
  if (*p == '-') { neg = 1; p++; }
  size_t len = strcspn(p, " \r\n");
  int nd = (int)((len + 7) / 8);
  uint32_t *d = (uint32_t *)calloc(nd ? nd : 1, sizeof(uint32_t));
  for (size_t i = 0; i < len; i++) {
    char ch = p[len - 1 - i];
    uint32_t v = (ch >= '0' && ch <= '9') ? (uint32_t)(ch - '0') : (uint32_t)((ch | 32) - 'a' + 10);
    d[i / 8] |= v << (4 * (i % 8));
  }
  while (nd > 0 && d[nd - 1] == 0) nd--;
  bn_from_io(r, neg ? -nd : nd, d);
  free(d);
  return 1;
}

static void print_hex(const bn *a) {
  if (a->n == 0) { printf("0"); return; }
  if (a->neg) printf("-");
  printf("%x", a->d[a->n - 1]);
  for (int i = a->n - 2; i >= 0; i--) printf("%08x", a->d[i]);
}

static int job_factor(void) {
  int N, K, g;
  if (!fgets(line, sizeof line, stdin) || sscanf(line, "%d %d %d", &N, &K, &g) != 3) return 2;
  bn *X = (bn *)calloc((size_t)2 * N - 1, sizeof(bn));
  int64_t total = 0;
  for (int i = 0; i < 2 * N - 1; i++) { bn_init(&X[i]); if (!read_hex(&X[i])) return 2; total += X[i].n; }
  int32_t *slen = (int32_t *)calloc((size_t)2 * N - 1, sizeof(int32_t));
  int64_t *off = (int64_t *)calloc((size_t)2 * N - 1, sizeof(int64_t));
  uint32_t *dig = (uint32_t *)calloc((size_t)(total ? total : 1), sizeof(uint32_t));
  int64_t pos = 0;
  for (int i = 0; i < 2 * N - 1; i++) {
    slen[i] = X[i].neg ? -X[i].n : X[i].n;
    off[i] = pos;
    if (X[i].n) memcpy(dig + pos, X[i].d, (size_t)X[i].n * 4);
    pos += X[i].n;
  }
  bn xs; bn_init(&xs);
  if (!read_hex(&xs)) return 2;
  hko_fact *f = hko_factor(N, K, slen, off, dig, xs.neg ? -xs.n : xs.n, xs.n ? xs.d : dig, 0, 2);
  if (!f) return 3;
  for (int pc = 0; pc < N; pc++)
    for (int r = pc; r < N; r++) { printf("C %d %d ", pc, r); print_hex(&f->C[tri_idx(N, pc, r)]); printf("\n"); }
  for (int pc = 0; pc + 1 < N; pc++)
    for (int r = pc + 1; r < N; r++) { printf("L %d %d ", pc, r); print_hex(&f->L[lidx(N, pc, r)]); printf("\n"); }
  hko_vec *b = hko_vec_new(N, NULL, NULL, NULL);
  for (int i = 0; i < N; i++) if (!read_hex(&b->v[i])) return 2;
  hko_vec *y = f->status == 0 ? hko_solve(f, b, 3, g) : NULL;
  if (y) {
    for (int i = 0; i < N; i++) { printf("Y %d ", i); print_hex(&y->v[i]); printf("\n"); }
    hko_vec_free(y);
  }
  hko_vec_free(b);
  hko_fact_free(f);
  for (int i = 0; i < 2 * N - 1; i++) bn_free(&X[i]);
  free(X); free(slen); free(off); free(dig); bn_free(&xs);
  return 0;
}

static int job_prim(void) {
  int op;
  long s;
  while (fgets(line, sizeof line, stdin)) {
    if (sscanf(line, "%d %ld", &op, &s) != 2) return 2;
    bn a, b;
    bn_init(&a); bn_init(&b);
    if (!read_hex(&a) || !read_hex(&b)) return 2;
    int64_t cap = a.n + b.n + (s > 0 ? s / 32 : 0) + 4;
    uint32_t *rd = (uint32_t *)calloc((size_t)cap, sizeof(uint32_t));
    int32_t rs = 0;
    int64_t n = hko_prim(op, a.neg ? -a.n : a.n, a.n ? a.d : rd, b.neg ? -b.n : b.n, b.n ? b.d : rd, s, &rs, rd, cap);
    if (n > cap) return 4;
    bn r; bn_init(&r);
    bn_from_io(&r, rs, rd);
    print_hex(&r);
    printf("\n");
    bn_free(&r); bn_free(&a); bn_free(&b); free(rd);
  }
  return 0;
}

int main(void) {
  if (!fgets(line, sizeof line, stdin)) return 2;
  if (!strncmp(line, "factor", 6)) return job_factor();
  if (!strncmp(line, "prim", 4)) return job_prim();
  return 2;
}
