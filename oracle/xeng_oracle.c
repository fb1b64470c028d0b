/*
 * CPU oracle of the X-engine.  TEST INFRASTRUCTURE ONLY: it is loaded by the
 * tests, by the smoke check and by the benchmark's CPU-baseline leg, never by
 * the product path.  It shares no code, header or table with the HIP library.
 *
 * What it computes (paper, Sec. 2 first paragraph and Sec. 2.2/2.3): for every
 * frequency channel, each pair of inputs is cross-multiplied at the same
 * frequency (the "X" of an FX correlator), a complex multiply-accumulate, and
 * the products are integrated over a chosen duration.  All pairs are formed,
 * auto-correlations included, in the natural order "fix one input, run over
 * all inputs up to and including itself" (Sec. 2.3).  Written out:
 *
 *     V[f][k(i,j)] = sum_t x_i(t,f) * conj(x_j(t,f)),   0 <= j <= i < N,
 *     k(i,j)       = i(i+1)/2 + j,
 *
 * i.e. with x = a + j b:  Re V = sum(a_i a_j + b_i b_j),
 *                         Im V = sum(b_i a_j - a_i b_j).
 *
 * Input samples (Sec. 2.1, equaliser, and Sec. 2.3, packet payload): one byte
 * per complex sample, a 4-bit two's-complement real part and a 4-bit
 * two's-complement imaginary part; the real part is read from the high nibble.
 * Layout [time][channel][input].
 *
 * Integer sums are kept in int64, so the integer function is exact for any
 * integration length this library is asked about; the float64 function has
 * the same loop structure and serves the FX == XF and delay checks.
 */
#include <stdint.h>
#include <stdlib.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* Two's-complement value of a 4-bit code (codes 8..15 are -8..-1). */
static int sext4(int code)
{
    return (code & 0x8) ? code - 16 : code;
}

void oracle_decode(uint8_t byte, int32_t *re, int32_t *im)
{
    *re = sext4((byte >> 4) & 0xF);
    *im = sext4(byte & 0xF);
}

int64_t oracle_nbaselines(int32_t n)
{
    return n < 0 ? -1 : (int64_t)n * (n + 1) / 2;
}

int64_t oracle_baseline_index(int32_t i, int32_t j)
{
    if (i < 0 || j < 0 || j > i) return -1;
    return (int64_t)i * (i + 1) / 2 + j;
}

/* Threads an OpenMP region of this library uses by default. */
int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

/*
 * acc[c][k][0..1] += sum over t of x_i conj(x_j) for channels f = f0 + c,
 * c in [0, f1 - f0).  v is uint8 [T][F][N].  Returns 0, or -1 on bad sizes.
 */
int oracle_accumulate_i4(const uint8_t *v, int64_t T, int32_t F, int32_t N,
                         int32_t f0, int32_t f1, int64_t *acc, int nthreads)
{
    if (T < 0 || F < 1 || N < 1 || f0 < 0 || f1 > F || f0 > f1) return -1;
    const int64_t nbl = oracle_nbaselines(N);
    set_threads(nthreads);
    #pragma omp parallel
    {
        int32_t *a = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
        int32_t *b = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
        #pragma omp for schedule(dynamic, 1)
        for (int32_t f = f0; f < f1; ++f) {
            int64_t *vf = acc + (int64_t)(f - f0) * nbl * 2;
            for (int64_t t = 0; t < T; ++t) {
                const uint8_t *row = v + (t * F + f) * (int64_t)N;
                for (int32_t n = 0; n < N; ++n) oracle_decode(row[n], &a[n], &b[n]);
                for (int32_t i = 0; i < N; ++i) {
                    int64_t *vi = vf + oracle_baseline_index(i, 0) * 2;
                    for (int32_t j = 0; j <= i; ++j) {
                        vi[2 * j]     += (int64_t)(a[i] * a[j] + b[i] * b[j]);
                        vi[2 * j + 1] += (int64_t)(b[i] * a[j] - a[i] * b[j]);
                    }
                }
            }
        }
        free(a);
        free(b);
    }
    return 0;
}

/*
 * Same definition on float64 complex samples: x is double [T][F][N][2]
 * (re, im), acc is double [F][nbl][2].
 */
int oracle_accumulate_c128(const double *x, int64_t T, int32_t F, int32_t N,
                           double *acc, int nthreads)
{
    if (T < 0 || F < 1 || N < 1) return -1;
    const int64_t nbl = oracle_nbaselines(N);
    set_threads(nthreads);
    #pragma omp parallel for schedule(dynamic, 1)
    for (int32_t f = 0; f < F; ++f) {
        double *vf = acc + (int64_t)f * nbl * 2;
        for (int64_t t = 0; t < T; ++t) {
            const double *row = x + (t * F + f) * (int64_t)N * 2;
            for (int32_t i = 0; i < N; ++i) {
                const double ai = row[2 * i], bi = row[2 * i + 1];
                double *vi = vf + oracle_baseline_index(i, 0) * 2;
                for (int32_t j = 0; j <= i; ++j) {
                    const double aj = row[2 * j], bj = row[2 * j + 1];
                    vi[2 * j]     += ai * aj + bi * bj;
                    vi[2 * j + 1] += bi * aj - ai * bj;
                }
            }
        }
    }
    return 0;
}

/* Narrow an int64 accumulator to int32; returns the count of values that do not fit. */
int64_t oracle_to_int32(const int64_t *acc, int64_t n, int32_t *out)
{
    int64_t bad = 0;
    for (int64_t k = 0; k < n; ++k) {
        if (acc[k] > INT32_MAX || acc[k] < INT32_MIN) { ++bad; out[k] = 0; }
        else out[k] = (int32_t)acc[k];
    }
    return bad;
}
