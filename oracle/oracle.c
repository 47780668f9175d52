/*
 * Correctness oracle for the sparse tensor algebra leaf kernels.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file: only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no header, helper or table with the
 * GPU library.
 *
 * Every operation is its plain definition in tensor index notation (paper,
 * Sec. II-A: every index variable is a loop, and a variable that appears only
 * on the right-hand side is summed over its whole domain), iterated over the
 * coordinate tree of the Dense/Compressed encoding (Sec. III-B: the
 * coordinates of parent entry i are stored at positions [pos[i], pos[i+1]) of
 * crd), in the same loop shape as the generated row-based SpMV leaf
 * (Fig. 8b, label (4)).  The six kernels are the ones defined in Sec. VI-A;
 * the inner product of two 3-tensors is the same notation with no free
 * index.
 *
 * Arithmetic: every input value is passed as an IEEE double (FP32 and BF16
 * inputs widen to double exactly).  All products and sums are carried out in
 * long double (x87, 64-bit significand) and rounded to double once on output.
 * Each output entry also reports S = sum of |term|, the magnitude that scales
 * the comparison tolerance of a reordered floating-point sum.
 *
 * Index arrays are int32 (pos and crd), sizes are int64.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef long double ld;

static ld ld_abs(ld v) { return v < 0 ? -v : v; }

/* ------------------------------------------------------------------------ */
/* SpMV  a(i) = B(i,j) * c(j)                (Sec. VI-A; leaf of Fig. 8b)    */
/* B is CSR = (Dense, Compressed).  If rows != NULL only those rows are      */
/* evaluated and the outputs are compacted (a[r], S[r] for r < nrows).       */
/* ------------------------------------------------------------------------ */
void orc_spmv(int64_t n, const int32_t *pos, const int32_t *crd,
              const double *vals, const double *c, const int64_t *rows,
              int64_t nrows, double *a, double *S)
{
    int64_t count = rows ? nrows : n;
    for (int64_t r = 0; r < count; ++r) {
        int64_t i = rows ? rows[r] : r;
        ld sum = 0.0L, mag = 0.0L;
        for (int64_t p = pos[i]; p < pos[i + 1]; ++p) {
            int64_t j = crd[p];
            ld term = (ld)vals[p] * (ld)c[j];
            sum += term;
            mag += ld_abs(term);
        }
        a[r] = (double)sum;
        if (S) S[r] = (double)mag;
    }
}

/* ------------------------------------------------------------------------ */
/* SpMM  A(i,j) = B(i,k) * C(k,j)                          (Sec. VI-A)       */
/* C is m x N row-major with leading dimension ldc; A is n x N row-major     */
/* with leading dimension lda (compacted rows when rows != NULL).            */
/* ------------------------------------------------------------------------ */
void orc_spmm(int64_t n, int64_t N, const int32_t *pos, const int32_t *crd,
              const double *vals, const double *C, int64_t ldc,
              const int64_t *rows, int64_t nrows, double *A, int64_t lda,
              double *S)
{
    int64_t count = rows ? nrows : n;
    ld *acc = (ld *)malloc(sizeof(ld) * (size_t)(N > 0 ? N : 1));
    ld *mag = (ld *)malloc(sizeof(ld) * (size_t)(N > 0 ? N : 1));
    for (int64_t r = 0; r < count; ++r) {
        int64_t i = rows ? rows[r] : r;
        for (int64_t j = 0; j < N; ++j) { acc[j] = 0.0L; mag[j] = 0.0L; }
        for (int64_t p = pos[i]; p < pos[i + 1]; ++p) {
            int64_t k = crd[p];
            for (int64_t j = 0; j < N; ++j) {
                ld term = (ld)vals[p] * (ld)C[k * ldc + j];
                acc[j] += term;
                mag[j] += ld_abs(term);
            }
        }
        for (int64_t j = 0; j < N; ++j) {
            A[r * lda + j] = (double)acc[j];
            if (S) S[r * lda + j] = (double)mag[j];
        }
    }
    free(acc);
    free(mag);
}

/* ------------------------------------------------------------------------ */
/* SpAdd3  A(i,j) = B(i,j) + C(i,j) + D(i,j)                (Sec. VI-A)      */
/* The output pattern is unknown in advance, so it is built in two phases    */
/* (Sec. V-B): a symbolic phase that counts the coordinates of every output  */
/* row, and a numeric phase that writes them.  The output keeps every        */
/* coordinate present in any operand (a structural union: a value that       */
/* cancels to zero is still stored).  Coordinates are strictly increasing    */
/* within a row.  A value sums the operands present, in the order B, C, D.   */
/* ------------------------------------------------------------------------ */
static int64_t union_row(const int32_t *c0, int64_t n0, const int32_t *c1,
                         int64_t n1, const int32_t *c2, int64_t n2,
                         const double *v0, const double *v1, const double *v2,
                         int32_t *out_crd, double *out_val, double *out_S)
{
    int64_t a = 0, b = 0, d = 0, k = 0;
    for (;;) {
        int64_t best = INT64_MAX;
        if (a < n0 && c0[a] < best) best = c0[a];
        if (b < n1 && c1[b] < best) best = c1[b];
        if (d < n2 && c2[d] < best) best = c2[d];
        if (best == INT64_MAX) break;
        ld sum = 0.0L, mag = 0.0L;
        int with_values = v0 != NULL;   /* NULL in the symbolic phase */
        if (a < n0 && c0[a] == best) {
            if (with_values) { sum += (ld)v0[a]; mag += ld_abs((ld)v0[a]); }
            ++a;
        }
        if (b < n1 && c1[b] == best) {
            if (with_values) { sum += (ld)v1[b]; mag += ld_abs((ld)v1[b]); }
            ++b;
        }
        if (d < n2 && c2[d] == best) {
            if (with_values) { sum += (ld)v2[d]; mag += ld_abs((ld)v2[d]); }
            ++d;
        }
        if (out_crd) out_crd[k] = (int32_t)best;
        if (out_val) out_val[k] = (double)sum;
        if (out_S) out_S[k] = (double)mag;
        ++k;
    }
    return k;
}

/* Symbolic phase: A_pos[0..n] and the output nonzero count (returned). */
int64_t orc_spadd3_symbolic(int64_t n,
                            const int32_t *Bp, const int32_t *Bc,
                            const int32_t *Cp, const int32_t *Cc,
                            const int32_t *Dp, const int32_t *Dc,
                            int32_t *A_pos)
{
    int64_t total = 0;
    A_pos[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t k = union_row(Bc + Bp[i], Bp[i + 1] - Bp[i],
                              Cc + Cp[i], Cp[i + 1] - Cp[i],
                              Dc + Dp[i], Dp[i + 1] - Dp[i],
                              NULL, NULL, NULL, NULL, NULL, NULL);
        total += k;
        A_pos[i + 1] = (int32_t)total;
    }
    return total;
}

/* Numeric phase: A_crd and A_vals at the positions the symbolic phase set. */
void orc_spadd3_numeric(int64_t n,
                        const int32_t *Bp, const int32_t *Bc, const double *Bv,
                        const int32_t *Cp, const int32_t *Cc, const double *Cv,
                        const int32_t *Dp, const int32_t *Dc, const double *Dv,
                        const int32_t *A_pos, int32_t *A_crd, double *A_vals,
                        double *A_S)
{
    for (int64_t i = 0; i < n; ++i) {
        int64_t o = A_pos[i];
        union_row(Bc + Bp[i], Bp[i + 1] - Bp[i],
                  Cc + Cp[i], Cp[i + 1] - Cp[i],
                  Dc + Dp[i], Dp[i + 1] - Dp[i],
                  Bv + Bp[i], Cv + Cp[i], Dv + Dp[i],
                  A_crd + o, A_vals + o, A_S ? A_S + o : NULL);
    }
}

/* ------------------------------------------------------------------------ */
/* SDDMM  A(i,j) = B(i,j) * C(i,k) * D(j,k)                 (Sec. VI-A)      */
/* The paper writes the last factor as D(k,j); here D is stored with one row */
/* per column coordinate j (row-major m x K), so D(j,k) is the same tensor   */
/* transposed.  The output keeps B's pattern (a pattern-preserving output,   */
/* Sec. V-B): A_vals[p] for every stored position p of B.                    */
/* ------------------------------------------------------------------------ */
void orc_sddmm(int64_t n, int64_t K, const int32_t *pos, const int32_t *crd,
               const double *Bv, const double *C, int64_t ldc,
               const double *D, int64_t ldd, double *A_vals, double *A_S)
{
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t p = pos[i]; p < pos[i + 1]; ++p) {
            int64_t j = crd[p];
            ld sum = 0.0L, mag = 0.0L;
            for (int64_t k = 0; k < K; ++k) {
                ld term = (ld)Bv[p] * (ld)C[i * ldc + k] * (ld)D[j * ldd + k];
                sum += term;
                mag += ld_abs(term);
            }
            A_vals[p] = (double)sum;
            if (A_S) A_S[p] = (double)mag;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* SpTTV  A(i,j) = B(i,j,k) * c(k)                          (Sec. VI-A)      */
/* B is CSF = (Dense, Compressed, Compressed): pos1/crd1 hold the (i -> j)   */
/* level, pos2/crd2 the (fiber -> k) level.  The output keeps the (i,j)      */
/* pattern of B (Sec. V-B), so only one value per fiber is produced.         */
/* ------------------------------------------------------------------------ */
void orc_spttv(int64_t I, const int32_t *pos1, const int32_t *pos2,
               const int32_t *crd2, const double *vals, const double *c,
               double *A_vals, double *A_S)
{
    for (int64_t i = 0; i < I; ++i) {
        for (int64_t f = pos1[i]; f < pos1[i + 1]; ++f) {
            ld sum = 0.0L, mag = 0.0L;
            for (int64_t p = pos2[f]; p < pos2[f + 1]; ++p) {
                ld term = (ld)vals[p] * (ld)c[crd2[p]];
                sum += term;
                mag += ld_abs(term);
            }
            A_vals[f] = (double)sum;
            if (A_S) A_S[f] = (double)mag;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* SpMTTKRP  A(i,l) = B(i,j,k) * C(j,l) * D(k,l)            (Sec. VI-A)      */
/* C is J x R, D is K x R, A is I x R, all row-major.  If rows != NULL only  */
/* those slices i are evaluated (compacted output).                          */
/* ------------------------------------------------------------------------ */
void orc_mttkrp(int64_t I, int64_t R, const int32_t *pos1, const int32_t *crd1,
                const int32_t *pos2, const int32_t *crd2, const double *vals,
                const double *C, int64_t ldc, const double *D, int64_t ldd,
                const int64_t *rows, int64_t nrows, double *A, int64_t lda,
                double *S)
{
    int64_t count = rows ? nrows : I;
    ld *acc = (ld *)malloc(sizeof(ld) * (size_t)(R > 0 ? R : 1));
    ld *mag = (ld *)malloc(sizeof(ld) * (size_t)(R > 0 ? R : 1));
    for (int64_t r = 0; r < count; ++r) {
        int64_t i = rows ? rows[r] : r;
        for (int64_t l = 0; l < R; ++l) { acc[l] = 0.0L; mag[l] = 0.0L; }
        for (int64_t f = pos1[i]; f < pos1[i + 1]; ++f) {
            int64_t j = crd1[f];
            for (int64_t p = pos2[f]; p < pos2[f + 1]; ++p) {
                int64_t k = crd2[p];
                for (int64_t l = 0; l < R; ++l) {
                    ld term = (ld)vals[p] * (ld)C[j * ldc + l] * (ld)D[k * ldd + l];
                    acc[l] += term;
                    mag[l] += ld_abs(term);
                }
            }
        }
        for (int64_t l = 0; l < R; ++l) {
            A[r * lda + l] = (double)acc[l];
            if (S) S[r * lda + l] = (double)mag[l];
        }
    }
    free(acc);
    free(mag);
}

/* ------------------------------------------------------------------------ */
/* Inner product  a = B(i,j,k) * C(i,j,k)  (no free index: all summed).      */
/* General form: co-iterate the two coordinate trees level by level; a term  */
/* exists only where both tensors store the coordinate.  Works for order 2   */
/* (pos2/crd2 == NULL: B is CSR) and order 3 (CSF).                          */
/* ------------------------------------------------------------------------ */
static void intersect_level(int64_t bb, int64_t be, int64_t cb, int64_t ce,
                            const int32_t *bcrd, const int32_t *ccrd,
                            int last, const int32_t *bpos2, const int32_t *cpos2,
                            const int32_t *bcrd2, const int32_t *ccrd2,
                            const double *bv, const double *cv,
                            ld *sum, ld *mag)
{
    int64_t a = bb, b = cb;
    while (a < be && b < ce) {
        if (bcrd[a] < ccrd[b]) { ++a; continue; }
        if (bcrd[a] > ccrd[b]) { ++b; continue; }
        if (last) {
            ld term = (ld)bv[a] * (ld)cv[b];
            *sum += term;
            *mag += ld_abs(term);
        } else {
            intersect_level(bpos2[a], bpos2[a + 1], cpos2[b], cpos2[b + 1],
                            bcrd2, ccrd2, 1, NULL, NULL, NULL, NULL,
                            bv, cv, sum, mag);
        }
        ++a;
        ++b;
    }
}

double orc_inner(int64_t I,
                 const int32_t *Bpos1, const int32_t *Bcrd1,
                 const int32_t *Bpos2, const int32_t *Bcrd2, const double *Bv,
                 const int32_t *Cpos1, const int32_t *Ccrd1,
                 const int32_t *Cpos2, const int32_t *Ccrd2, const double *Cv,
                 double *S)
{
    ld sum = 0.0L, mag = 0.0L;
    int order3 = Bpos2 != NULL;
    for (int64_t i = 0; i < I; ++i) {
        intersect_level(Bpos1[i], Bpos1[i + 1], Cpos1[i], Cpos1[i + 1],
                        Bcrd1, Ccrd1, !order3, Bpos2, Cpos2, Bcrd2, Ccrd2,
                        Bv, Cv, &sum, &mag);
    }
    if (S) *S = (double)mag;
    return (double)sum;
}

/* ------------------------------------------------------------------------ */
/* (Dense, Dense, Compressed) 3-tensors (Sec. III-B; the format the paper    */
/* uses for its "patents" tensor, Sec. VI).  A Dense level stores nothing:   */
/* under slice i every coordinate j in [0, J) is present, at position        */
/* i*J + j of the middle level.  Only the last level has pos2/crd2, indexed  */
/* by that position.  The loops below are the statements' loops over this    */
/* coordinate tree, with the Dense middle level iterated as a full range.    */
/* ------------------------------------------------------------------------ */

/* SpTTV A(i,j) = B(i,j,k) * c(k): one output per (i,j), A row-major I x J. */
void orc_spttv_ddc(int64_t I, int64_t J, const int32_t *pos2, const int32_t *crd2,
                   const double *vals, const double *c, double *A, double *A_S)
{
    for (int64_t i = 0; i < I; ++i) {
        for (int64_t j = 0; j < J; ++j) {
            int64_t f = i * J + j;
            ld sum = 0.0L, mag = 0.0L;
            for (int64_t p = pos2[f]; p < pos2[f + 1]; ++p) {
                ld term = (ld)vals[p] * (ld)c[crd2[p]];
                sum += term;
                mag += ld_abs(term);
            }
            A[f] = (double)sum;
            if (A_S) A_S[f] = (double)mag;
        }
    }
}

/* SpMTTKRP A(i,l) = B(i,j,k) * C(j,l) * D(k,l) with B in (Dense, Dense,    */
/* Compressed); rows != NULL evaluates only those slices (compacted).        */
void orc_mttkrp_ddc(int64_t I, int64_t J, int64_t R, const int32_t *pos2,
                    const int32_t *crd2, const double *vals, const double *C,
                    int64_t ldc, const double *D, int64_t ldd, const int64_t *rows,
                    int64_t nrows, double *A, int64_t lda, double *S)
{
    int64_t count = rows ? nrows : I;
    ld *acc = (ld *)malloc(sizeof(ld) * (size_t)(R > 0 ? R : 1));
    ld *mag = (ld *)malloc(sizeof(ld) * (size_t)(R > 0 ? R : 1));
    for (int64_t r = 0; r < count; ++r) {
        int64_t i = rows ? rows[r] : r;
        for (int64_t l = 0; l < R; ++l) { acc[l] = 0.0L; mag[l] = 0.0L; }
        for (int64_t j = 0; j < J; ++j) {
            int64_t f = i * J + j;
            for (int64_t p = pos2[f]; p < pos2[f + 1]; ++p) {
                int64_t k = crd2[p];
                for (int64_t l = 0; l < R; ++l) {
                    ld term = (ld)vals[p] * (ld)C[j * ldc + l] * (ld)D[k * ldd + l];
                    acc[l] += term;
                    mag[l] += ld_abs(term);
                }
            }
        }
        for (int64_t l = 0; l < R; ++l) {
            A[r * lda + l] = (double)acc[l];
            if (S) S[r * lda + l] = (double)mag[l];
        }
    }
    free(acc);
    free(mag);
}

/* Inner product of two 3-tensors of shape I x J x K whose middle levels may */
/* each be Dense (pos1 == NULL) or Compressed.  Co-iteration of the middle   */
/* level (Sec. IV-C): Dense with Dense visits every j; a Compressed side is  */
/* iterated and the Dense side located at i*J + j; two Compressed sides are  */
/* intersected.  The last levels are then intersected as for CSF.           */
double orc_inner3(int64_t I, int64_t J,
                  const int32_t *Bpos1, const int32_t *Bcrd1,
                  const int32_t *Bpos2, const int32_t *Bcrd2, const double *Bv,
                  const int32_t *Cpos1, const int32_t *Ccrd1,
                  const int32_t *Cpos2, const int32_t *Ccrd2, const double *Cv,
                  double *S)
{
    ld sum = 0.0L, mag = 0.0L;
    for (int64_t i = 0; i < I; ++i) {
        if (!Bpos1 && !Cpos1) {
            for (int64_t j = 0; j < J; ++j) {
                int64_t f = i * J + j;
                intersect_level(Bpos2[f], Bpos2[f + 1], Cpos2[f], Cpos2[f + 1], Bcrd2, Ccrd2,
                                1, NULL, NULL, NULL, NULL, Bv, Cv, &sum, &mag);
            }
        } else if (!Bpos1) {
            for (int64_t g = Cpos1[i]; g < Cpos1[i + 1]; ++g) {
                int64_t f = i * J + Ccrd1[g];
                intersect_level(Bpos2[f], Bpos2[f + 1], Cpos2[g], Cpos2[g + 1], Bcrd2, Ccrd2,
                                1, NULL, NULL, NULL, NULL, Bv, Cv, &sum, &mag);
            }
        } else if (!Cpos1) {
            for (int64_t f = Bpos1[i]; f < Bpos1[i + 1]; ++f) {
                int64_t g = i * J + Bcrd1[f];
                intersect_level(Bpos2[f], Bpos2[f + 1], Cpos2[g], Cpos2[g + 1], Bcrd2, Ccrd2,
                                1, NULL, NULL, NULL, NULL, Bv, Cv, &sum, &mag);
            }
        } else {
            intersect_level(Bpos1[i], Bpos1[i + 1], Cpos1[i], Cpos1[i + 1], Bcrd1, Ccrd1, 0,
                            Bpos2, Cpos2, Bcrd2, Ccrd2, Bv, Cv, &sum, &mag);
        }
    }
    if (S) *S = (double)mag;
    return (double)sum;
}

/* ------------------------------------------------------------------------ */
/* Universe partition of a Compressed level by coordinate value ranges       */
/* (Sec. III-A; Table I): each stored coordinate takes the color of the      */
/* range [bounds[c], bounds[c+1]) holding its value, and the preimage        */
/* through pos gives each row its positions of that color.  out[c*n + i] =   */
/* pos[i] + the number of coordinates of row i below bounds[c]; with sorted  */
/* coordinates, color c of row i is then [out[c*n+i], out[(c+1)*n+i]).        */
/* ------------------------------------------------------------------------ */
void orc_coord_partition(int64_t n, const int32_t *pos, const int32_t *crd, int64_t ncolors,
                         const int32_t *bounds, int32_t *out)
{
    for (int64_t c = 0; c <= ncolors; ++c) {
        for (int64_t i = 0; i < n; ++i) {
            int64_t below = 0;
            for (int64_t p = pos[i]; p < pos[i + 1]; ++p)
                if (crd[p] < bounds[c]) ++below;
            out[c * n + i] = (int32_t)(pos[i] + below);
        }
    }
}

/* SpMV over position windows: a(i) = sum over p in [begin[i], end[i]) of    */
/* vals[p] * c[crd[p]] (one color of the partition above).                  */
void orc_spmv_window(int64_t n, const int32_t *begin, const int32_t *end, const int32_t *crd,
                     const double *vals, const double *c, double *a, double *S)
{
    for (int64_t i = 0; i < n; ++i) {
        ld sum = 0.0L, mag = 0.0L;
        for (int64_t p = begin[i]; p < end[i]; ++p) {
            ld term = (ld)vals[p] * (ld)c[crd[p]];
            sum += term;
            mag += ld_abs(term);
        }
        a[i] = (double)sum;
        if (S) S[i] = (double)mag;
    }
}

/* ------------------------------------------------------------------------ */
/* Partitions of a Compressed level (Sec. III-A, IV-B, Table I).             */
/*                                                                           */
/* A tile of a leaf kernel is described by the pair (row, position) at which */
/* it starts: it covers positions [tile_pos[t], tile_pos[t+1]) and finishes  */
/* the rows [tile_row[t], tile_row[t+1]).  Row r is finished once all of its */
/* positions [pos[r], pos[r+1]) are covered; an empty row, and a row whose   */
/* last position is p-1, counts as finished at position p (so a tile that    */
/* starts at position p starts after every row ending at or before p).       */
/* ntiles+1 entries are written; the last is (n, nnz).                       */
/* ------------------------------------------------------------------------ */

/* Universe partition of the Dense row level in blocks of R rows, carried to */
/* the Compressed level by an image through pos (Table I, partitionFromParent). */
int64_t orc_row_split(int64_t n, const int32_t *pos, int64_t R,
                      int32_t *tile_row, int32_t *tile_pos)
{
    int64_t ntiles = n > 0 ? (n + R - 1) / R : 0;
    for (int64_t t = 0; t <= ntiles; ++t) {
        int64_t r = t * R < n ? t * R : n;
        tile_row[t] = (int32_t)r;
        tile_pos[t] = pos[r];
    }
    return ntiles;
}

/* Number of rows finished at position p: the rows whose segment ends at or  */
/* before p, counted by scanning every row (the preimage of [0, p) through   */
/* pos, Table I, partitionFromChild).                                        */
int64_t orc_rows_finished_at(int64_t n, const int32_t *pos, int64_t p)
{
    int64_t count = 0;
    for (int64_t i = 0; i < n; ++i)
        if (pos[i + 1] <= p) ++count;
    return count;
}

/* Non-zero partition of the fused (i,j) positions in blocks of T positions */
/* (Sec. II-B coordinate fusion and the tilde operator), with rows derived  */
/* by preimage.  Tile 0 starts at row 0 so that leading empty rows are      */
/* finished by it.                                                          */
int64_t orc_nnz_split(int64_t n, const int32_t *pos, int64_t T,
                      int32_t *tile_row, int32_t *tile_pos)
{
    int64_t nnz = pos[n];
    int64_t ntiles = nnz > 0 ? (nnz + T - 1) / T : 1;
    for (int64_t t = 0; t <= ntiles; ++t) {
        int64_t p = t * T < nnz ? t * T : nnz;
        if (t == ntiles) p = nnz;
        tile_pos[t] = (int32_t)p;
        tile_row[t] = (int32_t)(t == 0 ? 0 : orc_rows_finished_at(n, pos, p));
    }
    return ntiles;
}

/* Equal split of the merged sequence of row ends and positions (a          */
/* merge-path split) in blocks of Dm items.  The sequence is walked one item */
/* at a time: the next item is the end of the current row if that row's      */
/* segment ends at or before the next position, else the next position.     */
int64_t orc_merge_split(int64_t n, const int32_t *pos, int64_t Dm,
                        int32_t *tile_row, int32_t *tile_pos)
{
    int64_t nnz = pos[n];
    int64_t total = n + nnz;
    int64_t ntiles = total > 0 ? (total + Dm - 1) / Dm : 1;
    int64_t i = 0, p = 0, d = 0;
    tile_row[0] = 0;
    tile_pos[0] = 0;
    for (int64_t t = 1; t <= ntiles; ++t) {
        int64_t target = t * Dm < total ? t * Dm : total;
        while (d < target) {
            if (i < n && pos[i + 1] <= p) ++i;
            else ++p;
            ++d;
        }
        tile_row[t] = (int32_t)i;
        tile_pos[t] = (int32_t)p;
    }
    return ntiles;
}

/* Two-level split of a CSF tensor (Dense, Compressed, Compressed) for the  */
/* fused (i,j,k) positions: blocks of T positions, each snapped back to the  */
/* first fiber not finished at the block boundary, so that every fiber lies  */
/* in one tile; slices are then derived from fibers by the same preimage.    */
/* Writes ntiles+1 triples (slice, fiber, position); the last is             */
/* (I, F, nnz).                                                              */
int64_t orc_csf_split(int64_t I, const int32_t *pos1, const int32_t *pos2,
                      int64_t T, int32_t *tile_slice, int32_t *tile_fiber,
                      int32_t *tile_pos)
{
    int64_t F = pos1[I];
    int64_t nnz = pos2[F];
    int64_t ntiles = nnz > 0 ? (nnz + T - 1) / T : 1;
    for (int64_t t = 0; t <= ntiles; ++t) {
        int64_t p = t * T < nnz ? t * T : nnz;
        if (t == ntiles) p = nnz;
        int64_t f = t == 0 ? 0 : orc_rows_finished_at(F, pos2, p);
        tile_fiber[t] = (int32_t)f;
        tile_pos[t] = pos2[f];
        tile_slice[t] = (int32_t)(t == 0 ? 0 : orc_rows_finished_at(I, pos1, f));
    }
    return ntiles;
}

/* ------------------------------------------------------------------------ */
/* Transposition: the CSR arrays of B^T from those of B (n x m).            */
/* A CSC matrix is (Dense, Compressed) over the reversed dimension order     */
/* (Sec. II-B), so the CSR of A^T read as CSC is A; transposing it gives A's */
/* CSR.  Definition: column c of B^T's rows holds B's entries of column c in */
/* increasing row order -- each column's count, their running sum as tpos,   */
/* then one sweep over B's rows in order appending each entry to its         */
/* column.  Values are moved unchanged.                                      */
/* ------------------------------------------------------------------------ */
void orc_transpose(int64_t n, int64_t m, const int32_t *pos, const int32_t *crd,
                   const double *vals, int32_t *tpos, int32_t *tcrd, double *tvals)
{
    int64_t *next = (int64_t *)calloc((size_t)(m > 0 ? m : 1), sizeof(int64_t));
    for (int64_t c = 0; c <= m; ++c) tpos[c] = 0;
    for (int64_t p = 0; p < pos[n]; ++p) tpos[crd[p] + 1] += 1;
    for (int64_t c = 0; c < m; ++c) tpos[c + 1] += tpos[c];
    for (int64_t c = 0; c < m; ++c) next[c] = tpos[c];
    for (int64_t i = 0; i < n; ++i)
        for (int64_t p = pos[i]; p < pos[i + 1]; ++p) {
            int64_t q = next[crd[p]]++;
            tcrd[q] = (int32_t)i;
            tvals[q] = vals[p];
        }
    free(next);
}

/* ------------------------------------------------------------------------ */
/* SpMV of a CSC matrix  y(i) = A(i,j) * x(j)  with A n x m stored by       */
/* columns (cpos over the m columns, rows in crd): the plain definition,     */
/* every stored entry's term added to its row.                               */
/* ------------------------------------------------------------------------ */
void orc_csc_spmv(int64_t n, int64_t m, const int32_t *cpos, const int32_t *crd,
                  const double *vals, const double *x, double *y, double *S)
{
    ld *acc = (ld *)calloc((size_t)(n > 0 ? n : 1), sizeof(ld));
    ld *mag = (ld *)calloc((size_t)(n > 0 ? n : 1), sizeof(ld));
    for (int64_t j = 0; j < m; ++j)
        for (int64_t p = cpos[j]; p < cpos[j + 1]; ++p) {
            ld term = (ld)vals[p] * (ld)x[j];
            acc[crd[p]] += term;
            mag[crd[p]] += ld_abs(term);
        }
    for (int64_t i = 0; i < n; ++i) {
        y[i] = (double)acc[i];
        if (S) S[i] = (double)mag[i];
    }
    free(acc);
    free(mag);
}
