/*
 * FP64 reference for generalized matrix multiply, C = alpha*A*B + beta*C.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into liboracle.so, which is
 * loaded by the test-suite, by the smoke check and by the CPU-baseline leg of
 * the benchmark.  The GPU library never links, includes or calls it, and it
 * shares no source with the GPU library.
 *
 * What it computes (Tiramisu paper, Section I, the gemm problem statement):
 * C = alpha * A B + beta * C, where A is M x K, B is K x N and C is M x N.
 * The paper says nothing about storage order or degenerate arguments; the
 * reading taken here is row-major storage with a leading dimension equal to
 * the row stride in elements, and the reference-BLAS conventions:
 *   - beta == 0: the old C is never read (NaN or Inf in it do not propagate);
 *   - K == 0 or alpha == 0: the result is beta * C0 (A and B are not read);
 *   - M == 0 or N == 0: nothing is written.
 *
 * Method: the plain definition.  For each row i an FP64 accumulator row
 * acc[0..N) starts at zero; for k = 0..K-1 and j = 0..N-1,
 * acc[j] += A[i,k] * B[k,j]; then C[i,j] = alpha*acc[j] + beta*C0[i,j].
 * Rows are independent, so they are shared among OpenMP threads; nothing is
 * blocked, fused or reordered beyond that.
 *
 * The old C (C0) and the result (C) are separate arrays so that the caller
 * keeps its input.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Returns 0 on success, -1 on an invalid argument (negative size, short
 * leading dimension, or a null pointer that the call would dereference). */
int oracle_gemm_f64(int64_t M, int64_t N, int64_t K, double alpha,
                    const double* A, int64_t lda, const double* B, int64_t ldb,
                    double beta, const double* C0, int64_t ldc0,
                    double* C, int64_t ldc)
{
    if (M < 0 || N < 0 || K < 0) return -1;
    if (M == 0 || N == 0) return 0;
    if (ldc < N || !C) return -1;
    int use_ab = (K > 0 && alpha != 0.0);
    if (use_ab && (lda < K || ldb < N || !A || !B)) return -1;
    if (beta != 0.0 && (ldc0 < N || !C0)) return -1;

    int64_t i;
#pragma omp parallel for schedule(dynamic, 1)
    for (i = 0; i < M; ++i) {
        double* acc = (double*)calloc((size_t)N, sizeof(double));
        if (use_ab) {
            for (int64_t k = 0; k < K; ++k) {
                const double a = A[i * lda + k];
                const double* brow = B + k * ldb;
                for (int64_t j = 0; j < N; ++j) acc[j] += a * brow[j];
            }
        }
        for (int64_t j = 0; j < N; ++j) {
            double ab = use_ab ? alpha * acc[j] : 0.0;
            double c = (beta != 0.0) ? beta * C0[i * ldc0 + j] : 0.0;
            C[i * ldc + j] = ab + c;
        }
        free(acc);
    }
    return 0;
}

/* Number of threads an OpenMP parallel region of this library uses. */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
