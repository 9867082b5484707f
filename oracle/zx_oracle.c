/*
 * Plain, slow CPU oracle for the bit-packed GF(2) ZX path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links or calls
 * this file; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark use it.  It shares no code, header or table with the GPU library.
 *
 * Every routine is written for a reader who checks it against the paper by
 * eye: single-threaded loops over vertices, vertex pairs and matrix rows,
 * one bit at a time where that is clearer.  Paper references are to
 * "Tsim: Fast Universal Simulator for Quantum Error Correction" (arXiv
 * 2604.01059), appendix "ZX-Calculus / Rewrite rules".
 *
 * Representation (same conventions as the public header, restated here):
 *   adj    n x W uint64 rows, W = ceil(n/64); bit c of row r = word c/64,
 *          bit c%64; symmetric, zero diagonal; every entry is a Hadamard edge.
 *   k      int8 phase per spider in units of pi/4, kept in 0..7.
 *   alive  W-word bitmask of spiders still present.
 *   bnd    W-word bitmask of spiders that carry a boundary wire.
 *   scalar the diagram represents  omega^phase8 * sqrt(2)^pow_sqrt2 * D,
 *          omega = e^{i pi/4}; rewrites multiply in the factor they emit.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOMATCH (-2)

typedef struct {
  int64_t pow_sqrt2;  /* power of sqrt(2) */
  int32_t phase8;     /* power of omega = e^{i pi/4}, mod 8 */
  int32_t pad;
  int64_t fill_in;    /* Hadamard edges toggled on by rewrites */
} or_scalar;

/*
 * Parameterized Pauli spiders (the paper's Pauli boxes: a spider whose phase
 * carries an extra a*pi with a a parity of binary parameters; section on ZX
 * representation, and appendix "Rewrite rules", where the rules take phases
 * pi/2 + b*pi and a*pi with binary a, b).  Spider v's phase is
 *   k_v pi/4 + (p_v . f) pi,
 * p_v a row of pw 64-bit words over the parameters f.  A rewrite whose
 * scalar depends on the parameters records a phase-pair term
 * (k_alpha, k_beta, u, v): the factor h(k_alpha pi/4, k_beta pi/4; u.f, v.f)
 * of the parameterized evaluation appendix (equation phase_pair), so that
 * the diagram equals  omega^phase8 sqrt(2)^pow_sqrt2 prod_terms h * rest.
 */
typedef struct {
  int pw;            /* words per parameter row; 0 = no parameters */
  uint64_t* rows;    /* n x pw */
  int32_t* term_k;   /* cap x 2: k_alpha, k_beta */
  uint64_t* term_u;  /* cap x pw */
  uint64_t* term_v;  /* cap x pw */
  int32_t cap, n_terms;
} or_params;

static int prow_zero(const or_params* par, int v) {
  for (int q = 0; q < par->pw; ++q)
    if (par->rows[(size_t)v * par->pw + q]) return 0;
  return 1;
}
/* p_dst ^= p_src */
static void prow_xor(or_params* par, int dst, int src) {
  for (int q = 0; q < par->pw; ++q) par->rows[(size_t)dst * par->pw + q] ^= par->rows[(size_t)src * par->pw + q];
}
static int add_term(or_params* par, int ka, int kb, int su, int sv) {
  if (par->n_terms >= par->cap) return OR_EINVAL;
  const int t = par->n_terms++;
  par->term_k[2 * t] = ka;
  par->term_k[2 * t + 1] = kb;
  for (int q = 0; q < par->pw; ++q) {
    par->term_u[(size_t)t * par->pw + q] = su >= 0 ? par->rows[(size_t)su * par->pw + q] : 0;
    par->term_v[(size_t)t * par->pw + q] = sv >= 0 ? par->rows[(size_t)sv * par->pw + q] : 0;
  }
  return OR_OK;
}

/* ---------------------------------------------------------------- bits -- */

static int bit_get(const uint64_t* row, int c) {
  return (int)((row[c / 64] >> (c % 64)) & 1u);
}
static void bit_put(uint64_t* row, int c, int v) {
  uint64_t m = (uint64_t)1 << (c % 64);
  if (v) row[c / 64] |= m; else row[c / 64] &= ~m;
}
static uint64_t* row_of(uint64_t* adj, int W, int r) { return adj + (size_t)r * W; }
static const uint64_t* crow_of(const uint64_t* adj, int W, int r) { return adj + (size_t)r * W; }

static int mod8(int x) { return ((x % 8) + 8) % 8; }

/* Toggle the Hadamard edge {x, y}; returns 1 if the edge was present. */
static int toggle_edge(uint64_t* adj, int W, int x, int y) {
  int was = bit_get(row_of(adj, W, x), y);
  bit_put(row_of(adj, W, x), y, !was);
  bit_put(row_of(adj, W, y), x, !was);
  return was;
}

static int is_edge(const uint64_t* adj, int W, int x, int y) {
  return bit_get(crow_of(adj, W, x), y);
}

/* Interior spider: present and without a boundary wire. */
static int is_interior(const uint64_t* alive, const uint64_t* bnd, int v) {
  return bit_get(alive, v) && !bit_get(bnd, v);
}

static int neighbours(const uint64_t* adj, int n, int W, int u, int* out) {
  int c = 0;
  for (int x = 0; x < n; ++x)
    if (is_edge(adj, W, u, x)) out[c++] = x;
  return c;
}

static void delete_spider(uint64_t* adj, int n, int W, int8_t* k, uint64_t* alive, int u) {
  for (int x = 0; x < n; ++x)
    if (is_edge(adj, W, u, x)) toggle_edge(adj, W, u, x);
  bit_put(alive, u, 0);
  k[u] = 0;
}

/* ------------------------------------------------- local complementation -- */
/*
 * Local complementation rule (appendix, rewrite rules, equation
 * "local_comp"): an interior spider u with phase pi/2 + b*pi (k_u = 2 + 4b)
 * and neighbours N(u) is removed; every pair of neighbours has its Hadamard
 * edge complemented; each neighbour's phase drops by pi/2 + b*pi; the
 * diagram picks up e^{-i b pi/2} e^{i pi/4} sqrt(2)^{(n-1)(n-2)/2}, n = |N(u)|.
 *
 * The printed scalar is for neighbours with no edges among them.  When a
 * complemented pair already had an edge, the two parallel Hadamard edges
 * cancel to nothing at a cost of a factor 1/2, so each edge toggled off
 * subtracts 2 from the sqrt(2) power (reading of the rule for general
 * neighbourhoods; pinned by brute-force tensor evaluation in the tests).
 *
 * graph_only: only complement N(u) (the graph operation tau_u), keep u,
 * phases and scalar untouched.
 */
int or_local_comp(int n, int W, uint64_t* adj, int8_t* k, uint64_t* alive,
                  const uint64_t* bnd, int u, int graph_only, or_scalar* sc, or_params* par) {
  if (u < 0 || u >= n) return OR_EINVAL;
  if (!bit_get(alive, u)) return OR_ENOMATCH;
  if (!graph_only && (!is_interior(alive, bnd, u) || (k[u] != 2 && k[u] != 6)))
    return OR_ENOMATCH;
  int* nb = (int*)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
  int deg = neighbours(adj, n, W, u, nb);
  int64_t toggled_off = 0, pairs = 0;
  for (int a = 0; a < deg; ++a)
    for (int b = a + 1; b < deg; ++b) {
      toggled_off += toggle_edge(adj, W, nb[a], nb[b]);
      pairs += 1;
    }
  if (!graph_only) {
    int bpar = (k[u] - 2) / 4; /* b of the rule: 0 for pi/2, 1 for 3pi/2 */
    for (int a = 0; a < deg; ++a) k[nb[a]] = (int8_t)mod8(k[nb[a]] - k[u]);
    const int has_par = par && par->pw && !prow_zero(par, u);
    if (!has_par) {
      sc->phase8 = mod8(sc->phase8 + 1 - 2 * bpar);
    } else {
      /* u's phase is pi/2 + (bpar + p_u.f) pi: neighbours lose p_u.f pi too
       * (-x pi = x pi mod 2 pi), and the factor e^{-i b pi/2} with
       * b = bpar XOR (p_u.f) becomes a term: for bpar = 0 it is
       * h(pi, pi/2; p_u.f, 0) / (2i), for bpar = 1 it is
       * -i h(0, pi/2; p_u.f, 0) / 2 (h(pi, pi/2; a, 0) = 2i e^{-i a pi/2},
       * h(0, pi/2; a, 0) = 2 e^{i a pi/2}); both constants are
       * omega^{-2} / 2, so with e^{i pi/4}: phase8 - 1, pow_sqrt2 - 2. */
      for (int a = 0; a < deg; ++a) prow_xor(par, nb[a], u);
      if (add_term(par, bpar ? 0 : 4, 2, u, -1) != OR_OK) { free(nb); return OR_EINVAL; }
      sc->phase8 = mod8(sc->phase8 - 1);
      sc->pow_sqrt2 -= 2;
    }
    sc->pow_sqrt2 += (int64_t)(deg - 1) * (deg - 2) / 2 - 2 * toggled_off;
    sc->fill_in += pairs - toggled_off;
    if (par && par->pw) for (int q = 0; q < par->pw; ++q) par->rows[(size_t)u * par->pw + q] = 0;
    delete_spider(adj, n, W, k, alive, u);
  }
  free(nb);
  return OR_OK;
}

/* ------------------------------------------------------------------ pivot -- */
/*
 * Pivoting rule (appendix, rewrite rules, equation "pivoting"): adjacent
 * interior Pauli spiders u (phase a*pi) and v (phase b*pi) are removed.  The
 * other neighbours split into A = N(u) only, C = N(v) only, B = both.  Every
 * pair between two different classes has its edge complemented (the drawing
 * omits one A-C edge; the rule is the complete tripartite toggle).  Phases:
 * A gets +b*pi, C gets +a*pi, B gets +a*pi + b*pi + pi.  Scalar
 * e^{i a b pi} sqrt(2)^E; the paper leaves E undefined, the reading used here
 * is E = (|A|-1)(|C|-1) + |B|(|A|+|C|-2) - 2 * (edges toggled off), pinned by
 * brute-force tensor evaluation in the tests.
 *
 * graph_only: only the tripartite toggle; u, v, phases and scalar are kept.
 */
int or_pivot(int n, int W, uint64_t* adj, int8_t* k, uint64_t* alive,
             const uint64_t* bnd, int u, int v, int graph_only, or_scalar* sc, or_params* par) {
  if (u < 0 || u >= n || v < 0 || v >= n || u == v) return OR_EINVAL;
  if (!bit_get(alive, u) || !bit_get(alive, v) || !is_edge(adj, W, u, v)) return OR_ENOMATCH;
  if (!graph_only) {
    if (!is_interior(alive, bnd, u) || !is_interior(alive, bnd, v)) return OR_ENOMATCH;
    if ((k[u] != 0 && k[u] != 4) || (k[v] != 0 && k[v] != 4)) return OR_ENOMATCH;
  }
  int* A = (int*)malloc(sizeof(int) * (size_t)n);
  int* B = (int*)malloc(sizeof(int) * (size_t)n);
  int* C = (int*)malloc(sizeof(int) * (size_t)n);
  int na = 0, nbb = 0, nc = 0;
  for (int x = 0; x < n; ++x) {
    if (x == u || x == v) continue;
    int in_u = is_edge(adj, W, u, x), in_v = is_edge(adj, W, v, x);
    if (in_u && !in_v) A[na++] = x;
    else if (in_u && in_v) B[nbb++] = x;
    else if (!in_u && in_v) C[nc++] = x;
  }
  int64_t toggled_off = 0, pairs = 0;
  for (int i = 0; i < na; ++i)
    for (int j = 0; j < nc; ++j) { toggled_off += toggle_edge(adj, W, A[i], C[j]); pairs++; }
  for (int i = 0; i < na; ++i)
    for (int j = 0; j < nbb; ++j) { toggled_off += toggle_edge(adj, W, A[i], B[j]); pairs++; }
  for (int i = 0; i < nbb; ++i)
    for (int j = 0; j < nc; ++j) { toggled_off += toggle_edge(adj, W, B[i], C[j]); pairs++; }
  if (!graph_only) {
    int a = k[u] / 4, b = k[v] / 4;
    for (int i = 0; i < na; ++i) k[A[i]] = (int8_t)mod8(k[A[i]] + 4 * b);
    for (int j = 0; j < nc; ++j) k[C[j]] = (int8_t)mod8(k[C[j]] + 4 * a);
    for (int i = 0; i < nbb; ++i) k[B[i]] = (int8_t)mod8(k[B[i]] + 4 * a + 4 * b + 4);
    const int has_par = par && par->pw && (!prow_zero(par, u) || !prow_zero(par, v));
    if (!has_par) {
      sc->phase8 = mod8(sc->phase8 + 4 * a * b);
    } else {
      /* u = (a + p_u.f) pi, v = (b + p_v.f) pi: A gains p_v, C gains p_u,
       * B gains both; the factor (-1)^{(a + p_u.f)(b + p_v.f)} is the term
       * h(a pi, b pi; p_u.f, p_v.f) / 2 (h(0, 0; x, y) = 2 (-1)^{xy}). */
      for (int i = 0; i < na; ++i) prow_xor(par, A[i], v);
      for (int j = 0; j < nc; ++j) prow_xor(par, C[j], u);
      for (int i = 0; i < nbb; ++i) { prow_xor(par, B[i], u); prow_xor(par, B[i], v); }
      if (add_term(par, 4 * a, 4 * b, u, v) != OR_OK) { free(A); free(B); free(C); return OR_EINVAL; }
      sc->pow_sqrt2 -= 2;
    }
    sc->pow_sqrt2 += (int64_t)(na - 1) * (nc - 1) + (int64_t)nbb * (na + nc - 2) - 2 * toggled_off;
    sc->fill_in += pairs - toggled_off;
    if (par && par->pw)
      for (int q = 0; q < par->pw; ++q) par->rows[(size_t)u * par->pw + q] = par->rows[(size_t)v * par->pw + q] = 0;
    delete_spider(adj, n, W, k, alive, u);
    delete_spider(adj, n, W, k, alive, v);
  }
  free(A); free(B); free(C);
  return OR_OK;
}

/* --------------------------------------------------- simplification loop -- */
/*
 * Fixed point of the two rules (appendix, stabilizer decompositions: the
 * reduction stops when no interior pi/2 spider and no adjacent pair of
 * interior pi spiders remains).  The paper does not fix an order, so the
 * schedule is the canonical one of this library, in rounds:
 *
 *  LC rounds: scan spiders in ascending id; a spider joins the round if it
 *    is an LC candidate (interior, k in {2, 6}) and is not adjacent to a
 *    spider already chosen this round.  Apply the chosen rewrites in
 *    ascending order.  Repeat until a round chooses nothing.
 *  Pivot rounds: scan candidate edges (u < v, both interior with k in
 *    {0, 4}) in lexicographic order; an edge joins the round if u and v are
 *    distinct from, and not adjacent to, every spider of the edges already
 *    chosen.  Apply in order.  Repeat until a round chooses nothing.
 *
 * Pivots add 0 or 4 to phases, so no interior pi/2 spider can reappear once
 * the LC rounds are exhausted; the state reached is the rules' fixed point.
 * Trace entries: {round, rule (0 = LC, 1 = pivot), u, v (-1 for LC)}.
 */
typedef struct { int32_t round, rule, u, v; } or_trace;

static int lc_candidate(const uint64_t* alive, const uint64_t* bnd, const int8_t* k, int v) {
  return is_interior(alive, bnd, v) && (k[v] == 2 || k[v] == 6);
}
static int pauli_candidate(const uint64_t* alive, const uint64_t* bnd, const int8_t* k, int v) {
  return is_interior(alive, bnd, v) && (k[v] == 0 || k[v] == 4);
}

/* The same schedule stopped once max_rounds rounds (> 0) have been applied;
 * used to reach the intermediate states of a greedy run. */
int or_simplify_rounds(int n, int W, uint64_t* adj, int8_t* k, uint64_t* alive,
                       const uint64_t* bnd, or_scalar* sc, or_trace* trace, int trace_cap,
                       int* n_trace, int* n_rounds, int max_rounds, or_params* par) {
  int* sel = (int*)malloc(sizeof(int) * (size_t)(2 * n + 2));
  int nt = 0, round = 0;
  /* LC rounds */
  for (;;) {
    if (max_rounds > 0 && round >= max_rounds) break;
    int ns = 0;
    for (int u = 0; u < n; ++u) {
      if (!lc_candidate(alive, bnd, k, u)) continue;
      int ok = 1;
      for (int i = 0; i < ns; ++i)
        if (is_edge(adj, W, u, sel[i])) { ok = 0; break; }
      if (ok) sel[ns++] = u;
    }
    if (ns == 0) break;
    for (int i = 0; i < ns; ++i) {
      int rc = or_local_comp(n, W, adj, k, alive, bnd, sel[i], 0, sc, par);
      if (rc != OR_OK) { free(sel); return rc; }
      if (nt < trace_cap) { trace[nt].round = round; trace[nt].rule = 0; trace[nt].u = sel[i]; trace[nt].v = -1; }
      nt++;
    }
    round++;
  }
  /* pivot rounds */
  for (;;) {
    if (max_rounds > 0 && round >= max_rounds) break;
    int np = 0; /* pairs stored as sel[2i], sel[2i+1] */
    for (int u = 0; u < n; ++u) {
      if (!pauli_candidate(alive, bnd, k, u)) continue;
      for (int v = u + 1; v < n; ++v) {
        if (!pauli_candidate(alive, bnd, k, v) || !is_edge(adj, W, u, v)) continue;
        int ok = 1;
        for (int i = 0; i < 2 * np && ok; ++i) {
          int w = sel[i];
          if (w == u || w == v || is_edge(adj, W, u, w) || is_edge(adj, W, v, w)) ok = 0;
        }
        if (ok) { sel[2 * np] = u; sel[2 * np + 1] = v; np++; }
      }
    }
    if (np == 0) break;
    for (int i = 0; i < np; ++i) {
      int rc = or_pivot(n, W, adj, k, alive, bnd, sel[2 * i], sel[2 * i + 1], 0, sc, par);
      if (rc != OR_OK) { free(sel); return rc; }
      if (nt < trace_cap) { trace[nt].round = round; trace[nt].rule = 1; trace[nt].u = sel[2 * i]; trace[nt].v = sel[2 * i + 1]; }
      nt++;
    }
    round++;
  }
  free(sel);
  *n_trace = nt;
  *n_rounds = round;
  return OR_OK;
}

int or_simplify(int n, int W, uint64_t* adj, int8_t* k, uint64_t* alive,
                const uint64_t* bnd, or_scalar* sc, or_trace* trace, int trace_cap,
                int* n_trace, int* n_rounds) {
  return or_simplify_rounds(n, W, adj, k, alive, bnd, sc, trace, trace_cap, n_trace, n_rounds, 0, NULL);
}

/* ----------------------------------------------------- GF(2) elimination -- */
/*
 * Gauss-Jordan elimination over GF(2) (the paper reduces a binary matrix by
 * Gaussian elimination over F2 to keep a linearly independent basis; section
 * on detectors/observables, equation "detector_sampling" and the sentence
 * after it).  Column by column, left to right: take the lowest-index row at
 * or below the current row that has a 1 in this column, swap it into the
 * current row, and add it to every other row that has a 1 in this column.
 * The result is the reduced row echelon form.  rowops counts the row
 * additions.  Bits at or beyond n_cols must be zero.
 * piv[i] = pivot column of output row i (-1 for i >= rank).
 * T (optional, m x ceil(m/64) words): the same swaps and additions applied
 * to the identity, so that T * A_in = R.
 */
int or_gf2_rref(int m, int n_cols, int64_t ld, uint64_t* A, int32_t* piv,
                int32_t* rank, int64_t* rowops, uint64_t* T, int64_t ldt) {
  int nw = (n_cols + 63) / 64;
  if (m < 0 || n_cols < 0 || ld < nw) return OR_EINVAL;
  if (T) {
    for (int i = 0; i < m; ++i) {
      memset(T + (size_t)i * ldt, 0, sizeof(uint64_t) * (size_t)ldt);
      bit_put(T + (size_t)i * ldt, i, 1);
    }
  }
  uint64_t* tmp = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(ld > ldt ? ld : ldt) + 8);
  int cur = 0;
  int64_t ops = 0;
  for (int c = 0; c < n_cols && cur < m; ++c) {
    int r = -1;
    for (int i = cur; i < m; ++i)
      if (bit_get(A + (size_t)i * ld, c)) { r = i; break; }
    if (r < 0) continue;
    if (r != cur) {
      memcpy(tmp, A + (size_t)r * ld, sizeof(uint64_t) * (size_t)nw);
      memcpy(A + (size_t)r * ld, A + (size_t)cur * ld, sizeof(uint64_t) * (size_t)nw);
      memcpy(A + (size_t)cur * ld, tmp, sizeof(uint64_t) * (size_t)nw);
      if (T) {
        memcpy(tmp, T + (size_t)r * ldt, sizeof(uint64_t) * (size_t)ldt);
        memcpy(T + (size_t)r * ldt, T + (size_t)cur * ldt, sizeof(uint64_t) * (size_t)ldt);
        memcpy(T + (size_t)cur * ldt, tmp, sizeof(uint64_t) * (size_t)ldt);
      }
    }
    const uint64_t* prow = A + (size_t)cur * ld;
    for (int i = 0; i < m; ++i) {
      if (i == cur || !bit_get(A + (size_t)i * ld, c)) continue;
      uint64_t* row = A + (size_t)i * ld;
      for (int w = 0; w < nw; ++w) row[w] ^= prow[w];
      if (T) {
        uint64_t* trow = T + (size_t)i * ldt;
        const uint64_t* tp = T + (size_t)cur * ldt;
        for (int w = 0; w < ldt; ++w) trow[w] ^= tp[w];
      }
      ops++;
    }
    piv[cur] = c;
    cur++;
  }
  for (int i = cur; i < m; ++i) piv[i] = -1;
  *rank = cur;
  *rowops = ops;
  free(tmp);
  return OR_OK;
}

/*
 * The same elimination with the row additions of each column spread over
 * host threads (OpenMP); used only to time the oracle on all host cores.
 * Identical results: rows are independent within one column step.
 */
int or_gf2_rref_omp(int m, int n_cols, int64_t ld, uint64_t* A, int32_t* piv, int32_t* rank) {
  int nw = (n_cols + 63) / 64;
  if (m < 0 || n_cols < 0 || ld < nw) return OR_EINVAL;
  uint64_t* tmp = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)ld + 8);
  int cur = 0;
  for (int c = 0; c < n_cols && cur < m; ++c) {
    int r = -1;
    for (int i = cur; i < m; ++i)
      if (bit_get(A + (size_t)i * ld, c)) { r = i; break; }
    if (r < 0) continue;
    if (r != cur) {
      memcpy(tmp, A + (size_t)r * ld, sizeof(uint64_t) * (size_t)nw);
      memcpy(A + (size_t)r * ld, A + (size_t)cur * ld, sizeof(uint64_t) * (size_t)nw);
      memcpy(A + (size_t)cur * ld, tmp, sizeof(uint64_t) * (size_t)nw);
    }
    const uint64_t* prow = A + (size_t)cur * ld;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < m; ++i) {
      if (i == cur || !bit_get(A + (size_t)i * ld, c)) continue;
      uint64_t* row = A + (size_t)i * ld;
      for (int w = 0; w < nw; ++w) row[w] ^= prow[w];
    }
    piv[cur] = c;
    cur++;
  }
  for (int i = cur; i < m; ++i) piv[i] = -1;
  *rank = cur;
  free(tmp);
  return OR_OK;
}

/* ---------------------------------------------------- frontier extraction -- */
/*
 * Biadjacency between the output-attached spiders and the rest, the matrix a
 * circuit-extraction step eliminates: row j = spider attached to output j,
 * column c = spider id c, bit set when that spider has a Hadamard edge to a
 * spider c that is present and not itself attached to an output.  The matrix
 * is then brought to reduced row echelon form by or_gf2_rref (same pivot
 * rule, same row-addition count).
 */
int or_frontier(int n, int W, const uint64_t* adj, const uint64_t* alive,
                const int32_t* outputs, int q, uint64_t* M, int32_t* piv,
                int32_t* rank, int64_t* rowops) {
  uint64_t* outmask = (uint64_t*)calloc((size_t)W + 1, sizeof(uint64_t));
  for (int j = 0; j < q; ++j) {
    if (outputs[j] < 0 || outputs[j] >= n) { free(outmask); return OR_EINVAL; }
    bit_put(outmask, outputs[j], 1);
  }
  for (int j = 0; j < q; ++j) {
    uint64_t* row = M + (size_t)j * W;
    memset(row, 0, sizeof(uint64_t) * (size_t)W);
    for (int c = 0; c < n; ++c)
      if (is_edge(adj, W, outputs[j], c) && bit_get(alive, c) && !bit_get(outmask, c))
        bit_put(row, c, 1);
  }
  free(outmask);
  return or_gf2_rref(q, n, W, M, piv, rank, rowops, NULL, 0);
}

/* --------------------------------------------------- Pauli commutation -- */
/*
 * Commutation of Pauli strings stored as X and Z bit vectors (the paper's
 * two-bit encoding of a single-qubit Pauli: (1,0) = X, (1,1) = Y, (0,1) = Z,
 * (0,0) = I).  Two strings commute exactly when the symplectic form
 *   sum_q x_i[q] z_j[q] + z_i[q] x_j[q]   (mod 2)
 * is zero.  C[i][j] = that parity; rows i0..i1-1 are computed.
 */
void or_pauli_commute(int64_t n_paulis, int n_words, const uint64_t* X,
                      const uint64_t* Z, int64_t ldq, int64_t i0, int64_t i1,
                      uint64_t* C, int64_t ldc) {
  for (int64_t i = i0; i < i1; ++i) {
    uint64_t* crow = C + (size_t)(i - i0) * ldc;
    memset(crow, 0, sizeof(uint64_t) * (size_t)ldc);
    for (int64_t j = 0; j < n_paulis; ++j) {
      int parity = 0;
      for (int w = 0; w < n_words; ++w) {
        uint64_t s = (X[i * ldq + w] & Z[j * ldq + w]) ^ (Z[i * ldq + w] & X[j * ldq + w]);
        parity ^= __builtin_popcountll(s) & 1;
      }
      if (parity) crow[j / 64] |= (uint64_t)1 << (j % 64);
    }
  }
}

/* ------------------------------------------------ batched parities -- */
/*
 * Parities of many parameter subsets for many parameter settings at once
 * (appendix "Parameterized evaluation of Clifford ZX diagrams", equation
 * parities: a_k = XOR_i u_ki f_i, batched over settings l).  Row k of U
 * selects the parameters of parity k, row l of F is setting l, and
 *   C[k][l] = (sum_i U[k][i] F[l][i]) mod 2
 * for rows k = 0..m-1 and settings l = 0..n-1, over the first k_bits bits.
 */
void or_gf2_matmul(int64_t m, int64_t n, int k_bits, const uint64_t* U, int64_t ldu,
                   const uint64_t* F, int64_t ldf, uint64_t* C, int64_t ldc) {
  for (int64_t k = 0; k < m; ++k) {
    uint64_t* crow = C + (size_t)k * ldc;
    memset(crow, 0, sizeof(uint64_t) * (size_t)ldc);
    for (int64_t l = 0; l < n; ++l) {
      int parity = 0;
      for (int i = 0; i < k_bits; ++i)
        parity ^= bit_get(U + (size_t)k * ldu, i) & bit_get(F + (size_t)l * ldf, i);
      if (parity) crow[l / 64] |= (uint64_t)1 << (l % 64);
    }
  }
}

/* ------------------------------------------------- detector sampling -- */
/*
 * Shots of the detector/observable bits f = T e mod 2 (section on the
 * repetition-code example, equation detector_sampling; paragraph on
 * sampling detectors, equation dets-only and the text after it).  Column j
 * of T lists the f bits that error mechanism j flips (col_ptr / col_idx);
 * mechanism j fires independently with probability prob[j].
 *
 * As the paper describes (following Stim), firing mechanisms are found by
 * sampling the gap to the next one from a geometric distribution instead of
 * testing every mechanism.  Probabilities that differ per mechanism are
 * handled by thinning: gaps are drawn for the largest probability pmax, and
 * a mechanism so reached fires with probability prob[j] / pmax.
 *
 * Random numbers: SplitMix64 (Steele, Lea, Flood 2014), counter based.  The
 * t-th draw of shot s is mix64(seed + (s * 2^32 + t + 1) * GAMMA).  Per
 * candidate: one draw u for the gap, G = floor(ln(U) / ln(1 - pmax)) with
 * U = ((u >> 11) + 1) 2^-53 in (0, 1] (no gap draw when pmax = 1: G = 0);
 * then one draw v for the thinning: the mechanism fires iff
 * (v >> 11) < floor(prob[j] / pmax * 2^53).
 * Output: row s - shot0 of F holds the n_f bits of shot s.
 */
static uint64_t sm_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
static uint64_t sm_draw(uint64_t seed, uint64_t t) {
  return sm_mix(seed + (t + 1) * 0x9E3779B97F4A7C15ull);
}

int or_detector_sample(int n_err, int n_f, const int32_t* col_ptr, const int32_t* col_idx,
                       const double* prob, uint64_t seed, int64_t shot0, int64_t n_shots,
                       uint64_t* F, int64_t ldf) {
  double pmax = 0.0;
  for (int j = 0; j < n_err; ++j) {
    if (!(prob[j] >= 0.0 && prob[j] <= 1.0)) return OR_EINVAL;
    if (prob[j] > pmax) pmax = prob[j];
  }
  const double two53 = 9007199254740992.0;
  /* ln(1 - pmax) through log1p: log(1.0 - pmax) rounds to 0 for pmax below
   * 2^-53, which would make every gap -inf */
  const double log1m = log1p(-pmax);  /* -inf when pmax = 1 */
  for (int64_t i = 0; i < n_shots; ++i) {
    uint64_t* row = F + (size_t)i * ldf;
    memset(row, 0, sizeof(uint64_t) * (size_t)ldf);
    if (pmax == 0.0) continue;
    const uint64_t base = (uint64_t)(shot0 + i) << 32;
    uint64_t t = 0;
    int64_t pos = 0;
    for (;;) {
      int64_t gap = 0;
      if (pmax < 1.0) {
        const double U = (double)((sm_draw(seed, base + t++) >> 11) + 1) / two53;
        const double g = floor(log(U) / log1m);
        if (!(g < (double)(n_err - pos))) break;  /* also ends on a NaN quotient */
        gap = (int64_t)g;
      }
      pos += gap;
      if (pos >= n_err) break;
      const uint64_t thr = (uint64_t)(prob[pos] / pmax * two53);
      if ((sm_draw(seed, base + t++) >> 11) < thr)
        for (int q = col_ptr[pos]; q < col_ptr[pos + 1]; ++q) {
          const int b = col_idx[q];
          row[b / 64] ^= (uint64_t)1 << (b % 64);
        }
      pos += 1;
    }
  }
  (void)n_f;
  return OR_OK;
}
