/*
 * ps_oracle.c -- plain CPU reference for the Proportional Similarity (PS,
 * Czekanowski) metric of Joubert et al., "Parallel Accelerated Vector
 * Similarity Calculations for Genomics Applications" (arXiv 1705.08210).
 *
 * TEST INFRASTRUCTURE.  This file is the oracle that the HIP library is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header, table or
 * helper with the HIP path.
 *
 * Every value is evaluated from the definitions, in double precision, with
 * each sum taken in sequential field order q = 0, 1, ..., n_f-1.  No blocking,
 * no reordering, no fused shortcuts.  OpenMP is used only over independent
 * output tuples; each tuple's arithmetic is sequential.  Build without
 * -ffast-math so the compiler may not reassociate the sums.
 *
 * Indexing is 0-based.  Input matrix layout: vector i occupies
 * V[i*ld + q], q < n_f (the column-major n_f x n_v matrix of Section 3.1).
 * Element types: PSO_F32 (float), PSO_U8 (unsigned char), PSO_F64 (double).
 *
 * Readings of the paper taken here:
 *  - d = 0 (all-zero pair or triple): the metric is 0 (the paper leaves 0/0
 *    undefined; no shared mass means no similarity).
 *  - Outputs are the distinct tuples only: pairs i<j (Section 2.1 symmetry
 *    remark) and triples i<j<k (Section 2.2 symmetry remark).
 *  - Packed output orders (the library's layouts, written here as plain
 *    running counters so that they are defined by the loops themselves):
 *      2-way: for j = 1..n_v-1, for i = 0..j-1            (colex order)
 *      3-way: for j = 1..n_v-2, for k = j+1..n_v-1, for i = 0..j-1
 *             (middle index j outermost: "j-slab" order)
 *  - c3 = (3 * n3) / (2 * d3), one double division.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { PSO_F32 = 0, PSO_U8 = 2, PSO_F64 = 3 };

/* Element q of vector i, widened exactly to double. */
static double elem(const void* V, int dt, int64_t ld, int64_t i, int64_t q) {
    int64_t at = i * ld + q;
    switch (dt) {
    case PSO_F32: return (double)((const float*)V)[at];
    case PSO_U8:  return (double)((const unsigned char*)V)[at];
    default:      return ((const double*)V)[at];
    }
}

static double min2(double a, double b) { return a < b ? a : b; }

int ps_oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void ps_oracle_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Per-vector sums s_i = sum_q v_{i,q}.  These are the pieces of the
 * denominators d2 = s_i + s_j (Section 2.1) and d3 = s_i + s_j + s_k
 * (Section 2.2). */
void ps_oracle_sums(const void* V, int dt, int64_t n_f, int64_t n_v,
                    int64_t ld, double* s) {
    for (int64_t i = 0; i < n_v; ++i) {
        double acc = 0.0;
        for (int64_t q = 0; q < n_f; ++q) acc += elem(V, dt, ld, i, q);
        s[i] = acc;
    }
}

/* 2-way numerator n2(v_i, v_j) = sum_q min(v_{i,q}, v_{j,q})
 * (Section 2.1, the "min-product"). */
double ps_oracle_n2(const void* V, int dt, int64_t n_f, int64_t ld,
                    int64_t i, int64_t j) {
    double acc = 0.0;
    for (int64_t q = 0; q < n_f; ++q)
        acc += min2(elem(V, dt, ld, i, q), elem(V, dt, ld, j, q));
    return acc;
}

/* 3-way term n3'(v_i, v_j, v_k) = sum_q min(v_{i,q}, v_{j,q}, v_{k,q})
 * (Section 2.2, the term subtracted in Eq. 1). */
double ps_oracle_n3p(const void* V, int dt, int64_t n_f, int64_t ld,
                     int64_t i, int64_t j, int64_t k) {
    double acc = 0.0;
    for (int64_t q = 0; q < n_f; ++q)
        acc += min2(min2(elem(V, dt, ld, i, q), elem(V, dt, ld, j, q)),
                    elem(V, dt, ld, k, q));
    return acc;
}

/* c2 = 2 n2 / d2 with d2 = s_i + s_j (Section 2.1); 0 when d2 = 0. */
static double c2_of(double n2, double si, double sj) {
    double d2 = si + sj;
    return d2 > 0.0 ? (2.0 * n2) / d2 : 0.0;
}

/* c3 = (3/2) n3 / d3 with n3 from Eq. 1 and d3 = s_i + s_j + s_k
 * (Section 2.2); 0 when d3 = 0. */
static double c3_of(double n2ij, double n2ik, double n2jk, double n3p,
                    double si, double sj, double sk) {
    double n3 = ((n2ij + n2ik) + n2jk) - n3p;
    double d3 = (si + sj) + sk;
    return d3 > 0.0 ? (3.0 * n3) / (2.0 * d3) : 0.0;
}

/* All pairs i<j, colex order.  c2 has n_v(n_v-1)/2 entries; n2 (optional)
 * receives the raw numerators in the same order. */
void ps_oracle_c2_all(const void* V, int dt, int64_t n_f, int64_t n_v,
                      int64_t ld, double* c2, double* n2) {
    double* s = (double*)malloc(sizeof(double) * (size_t)(n_v > 0 ? n_v : 1));
    ps_oracle_sums(V, dt, n_f, n_v, ld, s);
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = 1; j < n_v; ++j) {
        int64_t idx = j * (j - 1) / 2;  /* pairs with larger index < j */
        for (int64_t i = 0; i < j; ++i, ++idx) {
            double num = ps_oracle_n2(V, dt, n_f, ld, i, j);
            if (n2) n2[idx] = num;
            c2[idx] = c2_of(num, s[i], s[j]);
        }
    }
    free(s);
}

/* Listed pairs (I[t], J[t]), any order of the two indices.  s must hold
 * the per-vector sums (from ps_oracle_sums). */
void ps_oracle_c2_pairs(const void* V, int dt, int64_t n_f, int64_t ld,
                        const double* s, const int64_t* I, const int64_t* J,
                        int64_t n, double* c2, double* n2) {
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t t = 0; t < n; ++t) {
        double num = ps_oracle_n2(V, dt, n_f, ld, I[t], J[t]);
        if (n2) n2[t] = num;
        c2[t] = c2_of(num, s[I[t]], s[J[t]]);
    }
}

/* All triples i<j<k in j-slab order (j outermost, then k, then i).
 * c3 has n_v(n_v-1)(n_v-2)/6 entries.  The three n2 terms of Eq. 1 come
 * from a table of all pair numerators, as the paper describes ("table
 * lookup"). */
void ps_oracle_c3_all(const void* V, int dt, int64_t n_f, int64_t n_v,
                      int64_t ld, double* c3) {
    double* s = (double*)malloc(sizeof(double) * (size_t)(n_v > 0 ? n_v : 1));
    double* N2 = (double*)calloc((size_t)(n_v > 0 ? n_v * n_v : 1), sizeof(double));
    ps_oracle_sums(V, dt, n_f, n_v, ld, s);
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = 0; j < n_v; ++j)
        for (int64_t i = 0; i < j; ++i) {
            double num = ps_oracle_n2(V, dt, n_f, ld, i, j);
            N2[i * n_v + j] = num;
            N2[j * n_v + i] = num;
        }
    /* offset of the first triple of slab j: number of triples with a
     * smaller middle index, i.e. sum over t<j of t*(n_v-1-t) */
    int64_t* off = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_v > 0 ? n_v : 1));
    int64_t run = 0;
    for (int64_t j = 0; j < n_v; ++j) {
        off[j] = run;
        run += j * (n_v - 1 - j);
    }
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = 1; j < n_v - 1; ++j) {
        int64_t idx = off[j];
        for (int64_t k = j + 1; k < n_v; ++k)
            for (int64_t i = 0; i < j; ++i, ++idx) {
                double n3p = ps_oracle_n3p(V, dt, n_f, ld, i, j, k);
                c3[idx] = c3_of(N2[i * n_v + j], N2[i * n_v + k],
                                N2[j * n_v + k], n3p, s[i], s[j], s[k]);
            }
    }
    free(off);
    free(N2);
    free(s);
}

/* Listed triples (I[t], J[t], K[t]), pairwise distinct, any order.  Each n2
 * term is computed directly.  s must hold the per-vector sums.  n3 (optional)
 * receives the Eq. 1 numerators. */
void ps_oracle_c3_triples(const void* V, int dt, int64_t n_f, int64_t ld,
                          const double* s, const int64_t* I, const int64_t* J,
                          const int64_t* K, int64_t n, double* c3, double* n3) {
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < n; ++t) {
        int64_t i = I[t], j = J[t], k = K[t];
        double nij = ps_oracle_n2(V, dt, n_f, ld, i, j);
        double nik = ps_oracle_n2(V, dt, n_f, ld, i, k);
        double njk = ps_oracle_n2(V, dt, n_f, ld, j, k);
        double n3p = ps_oracle_n3p(V, dt, n_f, ld, i, j, k);
        if (n3) n3[t] = ((nij + nik) + njk) - n3p;
        c3[t] = c3_of(nij, nik, njk, n3p, s[i], s[j], s[k]);
    }
}
