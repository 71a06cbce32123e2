/*
 * Exact squared Euclidean distance transform on a pixel grid (test oracle).
 *
 * TEST INFRASTRUCTURE ONLY: built for the CPU oracle, never linked into the
 * HIP library.
 *
 * Role in the paper: the signed distance function of Sec. II-A (distance of a
 * pixel to the mask boundary) and its truncation (TSDF, Sec. III-A), computed
 * in the paper by the CUDA_TSDF routine of Alg. 1.  The distance is measured
 * between pixel centres: for every pixel p, D(p) = min over pixels q of the
 * feature class of |p - q|^2.
 *
 * Method: the two-phase separable transform of Meijster, Roerdink and
 * Hesselink (2000), in 64-bit integers.  Phase one gives, per column, the
 * distance to the nearest feature pixel in that column; phase two takes, per
 * row, the lower envelope of the parabolas (x - i)^2 + g(i)^2.  A column with
 * no feature carries the finite stand-in g = 4N, whose parabola can never beat
 * a real one (2 (N-1)^2 < 16 N^2); a pixel whose minimum is still >= 16 N^2
 * has no feature at all and gets -1.
 */
#include <stdint.h>
#include <stdlib.h>

static int64_t sq(int64_t v) { return v * v; }

/* cls: N*N bytes (0/1), row-major [y][x]; feature = pixels with cls == want.
 * out: N*N int64 squared distances, -1 where the feature set is empty. */
int oracle_sqedt(const uint8_t *cls, int N, int want, int64_t *out)
{
    if (N <= 0) return -1;
    const int64_t ginf = 4 * (int64_t)N;
    const int64_t none_at = 16 * (int64_t)N * (int64_t)N;
    int64_t *g = (int64_t *)malloc(sizeof(int64_t) * (size_t)N * (size_t)N);
    int64_t *s = (int64_t *)malloc(sizeof(int64_t) * (size_t)N);
    int64_t *t = (int64_t *)malloc(sizeof(int64_t) * (size_t)N);
    if (!g || !s || !t) { free(g); free(s); free(t); return -2; }

    /* phase one: nearest feature in the same column, scanning down then up */
    for (int x = 0; x < N; ++x) {
        g[x] = (cls[x] == want) ? 0 : ginf;
        for (int y = 1; y < N; ++y) {
            int64_t prev = g[(size_t)(y - 1) * N + x];
            g[(size_t)y * N + x] = (cls[(size_t)y * N + x] == want) ? 0
                                   : (prev >= ginf ? ginf : prev + 1);
        }
        for (int y = N - 2; y >= 0; --y) {
            int64_t below = g[(size_t)(y + 1) * N + x];
            if (below + 1 < g[(size_t)y * N + x]) g[(size_t)y * N + x] = below + 1;
        }
    }

    /* phase two: per row, lower envelope of (u - i)^2 + g(i)^2 */
    for (int y = 0; y < N; ++y) {
        const int64_t *gr = g + (size_t)y * N;
        int q = 0;
        s[0] = 0;
        t[0] = 0;
        for (int u = 1; u < N; ++u) {
            /* pop segments whose start is won by u */
            while (q >= 0 && sq(t[q] - s[q]) + sq(gr[s[q]]) > sq(t[q] - u) + sq(gr[u]))
                --q;
            if (q < 0) {
                q = 0;
                s[0] = u;
            } else {
                /* last position where s[q] is no worse than u */
                int64_t i = s[q];
                int64_t sep = (sq(u) - sq(i) + sq(gr[u]) - sq(gr[i])) / (2 * (u - i));
                int64_t w = 1 + sep;
                if (w < N) {
                    ++q;
                    s[q] = u;
                    t[q] = w;
                }
            }
        }
        for (int u = N - 1; u >= 0; --u) {
            int64_t d = sq(u - s[q]) + sq(gr[s[q]]);
            out[(size_t)y * N + u] = (d >= none_at) ? -1 : d;
            if (u == t[q]) --q;
        }
    }
    free(g);
    free(s);
    free(t);
    return 0;
}
