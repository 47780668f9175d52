/*
 * CPU comparison baseline for the benchmark (test infrastructure, not the
 * parity oracle): the SpMV and SpMM leaves as plain double-precision loops
 * over CSR rows, parallelized with OpenMP and dynamic load balance over
 * blocks of 1,024 rows, the form of the paper's CPU leaf (Sec. VI-A: an
 * OpenMP leaf with dynamic scheduling).  Inputs as the oracle takes them:
 * int32 pos/crd, double values and dense operands (row-major, leading
 * dimension ldc / lda).  Shares no code with the GPU library.
 *
 * Built by oracle.build() with gcc -O2 -fopenmp (no fast-math).
 */
#include <stdint.h>

#ifdef _OPENMP
#include <omp.h>
#endif

int cpu_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* a(i) = sum over p in row i of vals[p] * c[crd[p]] */
void cpu_spmv(int64_t n, const int32_t *pos, const int32_t *crd, const double *vals,
              const double *c, double *a)
{
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < n; ++i) {
        double sum = 0.0;
        for (int64_t p = pos[i]; p < pos[i + 1]; ++p)
            sum += vals[p] * c[crd[p]];
        a[i] = sum;
    }
}

/* A(i,:) = sum over p in row i of vals[p] * C(crd[p], :), N columns */
void cpu_spmm(int64_t n, int64_t N, const int32_t *pos, const int32_t *crd, const double *vals,
              const double *C, int64_t ldc, double *A, int64_t lda)
{
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < n; ++i) {
        double *out = A + i * lda;
        for (int64_t j = 0; j < N; ++j) out[j] = 0.0;
        for (int64_t p = pos[i]; p < pos[i + 1]; ++p) {
            const double v = vals[p];
            const double *row = C + (int64_t)crd[p] * ldc;
            for (int64_t j = 0; j < N; ++j) out[j] += v * row[j];
        }
    }
}
