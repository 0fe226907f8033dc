/*
 * Metropolis Monte Carlo sampler of the Gibbs-Boltzmann distribution
 * P(Q) ~ exp(-U(Q) / kT) of N particles in a periodic cubic box interacting
 * with the WCA pair potential of Sec. IV.A, Eq. (WCA), and the radial
 * distribution function g(r) of the samples.
 *
 * TEST INFRASTRUCTURE ONLY: the independent reference that the equilibrium
 * structure produced by the GPU time stepper is compared with (Sec. IV.A,
 * Table RDF). It shares nothing with the HIP path. Only tests, the smoke
 * check and the CPU-baseline leg of the benchmark may load it.
 *
 * Method: single-particle trial moves uniform in a cube of side 2 delta,
 * accepted with probability min(1, exp(-dU / kT)) (Metropolis et al., 1953);
 * pair energies through a linked cell list with cells at least one cutoff
 * wide; minimum-image distances. Random numbers: xoshiro256** seeded by
 * splitmix64 (Blackman and Vigna), doubles from the top 53 bits.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    uint64_t s[4];
} rng_t;

static uint64_t splitmix64(uint64_t* x) {
    uint64_t z = (*x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

static uint64_t next_u64(rng_t* r) {
    const uint64_t result = rotl(r->s[1] * 5, 7) * 9;
    const uint64_t t = r->s[1] << 17;
    r->s[2] ^= r->s[0];
    r->s[3] ^= r->s[1];
    r->s[1] ^= r->s[2];
    r->s[0] ^= r->s[3];
    r->s[2] ^= t;
    r->s[3] = rotl(r->s[3], 45);
    return result;
}

static double uniform(rng_t* r) { return (double)(next_u64(r) >> 11) * 0x1.0p-53; }

typedef struct {
    int n;
    double L, eps, sigma, rc2, kT;
    double* x;   /* n x 3 positions in [0, L) */
    int nc;      /* cells per axis */
    double csz;  /* cell side */
    int* head;   /* first particle of each cell, -1: empty */
    int* next;   /* doubly linked lists */
    int* prev;
    int* cell;
} sys_t;

/* WCA: 4 eps ((s/r)^12 - (s/r)^6) + eps inside r_c = 2^(1/6) sigma. */
static double wca(const sys_t* S, double r2) {
    if (r2 >= S->rc2) return 0.0;
    const double s2 = S->sigma * S->sigma / r2;
    const double s6 = s2 * s2 * s2;
    return 4.0 * S->eps * (s6 * s6 - s6) + S->eps;
}

static double min_image(double d, double L) {
    if (d > 0.5 * L) return d - L;
    if (d < -0.5 * L) return d + L;
    return d;
}

static int cell_of(const sys_t* S, const double* p) {
    int c[3];
    for (int a = 0; a < 3; ++a) {
        c[a] = (int)(p[a] / S->csz);
        if (c[a] >= S->nc) c[a] = S->nc - 1;
        if (c[a] < 0) c[a] = 0;
    }
    return (c[2] * S->nc + c[1]) * S->nc + c[0];
}

static void insert(sys_t* S, int i, int c) {
    S->cell[i] = c;
    S->prev[i] = -1;
    S->next[i] = S->head[c];
    if (S->head[c] >= 0) S->prev[S->head[c]] = i;
    S->head[c] = i;
}

static void unlink_particle(sys_t* S, int i) {
    const int c = S->cell[i];
    if (S->prev[i] >= 0)
        S->next[S->prev[i]] = S->next[i];
    else
        S->head[c] = S->next[i];
    if (S->next[i] >= 0) S->prev[S->next[i]] = S->prev[i];
}

/* Energy of particle i placed at p with every other particle. */
static double energy_at(const sys_t* S, int i, const double* p) {
    double e = 0.0;
    const int c = cell_of(S, p);
    const int cx = c % S->nc, cy = (c / S->nc) % S->nc, cz = c / (S->nc * S->nc);
    /* with fewer than three cells per axis a neighbour cell would be visited
       twice: then scan every particle */
    if (S->nc < 3) {
        for (int j = 0; j < S->n; ++j) {
            if (j == i) continue;
            double r2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                const double d = min_image(p[a] - S->x[3 * j + a], S->L);
                r2 += d * d;
            }
            e += wca(S, r2);
        }
        return e;
    }
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const int nx = (cx + dx + S->nc) % S->nc, ny = (cy + dy + S->nc) % S->nc,
                          nz = (cz + dz + S->nc) % S->nc;
                for (int j = S->head[(nz * S->nc + ny) * S->nc + nx]; j >= 0; j = S->next[j]) {
                    if (j == i) continue;
                    double r2 = 0.0;
                    for (int a = 0; a < 3; ++a) {
                        const double d = min_image(p[a] - S->x[3 * j + a], S->L);
                        r2 += d * d;
                    }
                    e += wca(S, r2);
                }
            }
    return e;
}

static void accumulate_gr(const sys_t* S, double rmax, int nbins, double* hist) {
    const double dr = rmax / nbins;
    for (int i = 0; i < S->n; ++i)
        for (int j = i + 1; j < S->n; ++j) {
            double r2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                const double d = min_image(S->x[3 * i + a] - S->x[3 * j + a], S->L);
                r2 += d * d;
            }
            if (r2 < rmax * rmax) {
                const int b = (int)(sqrt(r2) / dr);
                if (b < nbins) hist[b] += 1.0;
            }
        }
}

/*
 * Sample g(r).
 *   n, L: particle count and box side (rmax must not exceed L / 2)
 *   eps, sigma, kT: WCA strength and diameter, temperature
 *   x: n x 3 initial positions in [0, L) (overwritten with the final ones)
 *   delta: half side of the trial-move cube
 *   n_equil, n_sweeps: sweeps (n trial moves each) before and during sampling
 *   every: sweeps between samples of g(r)
 *   seed: random seed
 *   rmax, nbins, gr: g(r) on nbins bins of [0, rmax), normalised by the
 *       ideal-gas pair count of each spherical shell
 *   acceptance: fraction of accepted moves during sampling (may be NULL)
 * Returns 0, or -1 on invalid arguments / allocation failure.
 */
int mc_wca_gr(int n, double L, double eps, double sigma, double kT, double* x, double delta, long long n_equil,
              long long n_sweeps, int every, uint64_t seed, double rmax, int nbins, double* gr,
              double* acceptance) {
    if (n < 2 || !(L > 0) || !(kT > 0) || !(sigma > 0) || nbins < 1 || !(rmax > 0) || rmax > 0.5 * L || every < 1)
        return -1;
    sys_t S;
    memset(&S, 0, sizeof(S));
    S.n = n;
    S.L = L;
    S.eps = eps;
    S.sigma = sigma;
    S.rc2 = pow(2.0, 1.0 / 3.0) * sigma * sigma;
    S.kT = kT;
    S.x = x;
    S.nc = (int)floor(L / sqrt(S.rc2));
    if (S.nc < 1) S.nc = 1;
    S.csz = L / S.nc;
    const int ncell = S.nc * S.nc * S.nc;
    S.head = (int*)malloc(sizeof(int) * (size_t)ncell);
    S.next = (int*)malloc(sizeof(int) * (size_t)n);
    S.prev = (int*)malloc(sizeof(int) * (size_t)n);
    S.cell = (int*)malloc(sizeof(int) * (size_t)n);
    double* hist = (double*)calloc((size_t)nbins, sizeof(double));
    if (!S.head || !S.next || !S.prev || !S.cell || !hist) {
        free(S.head); free(S.next); free(S.prev); free(S.cell); free(hist);
        return -1;
    }
    for (int c = 0; c < ncell; ++c) S.head[c] = -1;
    for (int i = 0; i < n; ++i) {
        for (int a = 0; a < 3; ++a) {
            double v = fmod(x[3 * i + a], L);
            if (v < 0) v += L;
            x[3 * i + a] = v;
        }
        insert(&S, i, cell_of(&S, x + 3 * i));
    }
    rng_t R;
    uint64_t sm = seed;
    for (int k = 0; k < 4; ++k) R.s[k] = splitmix64(&sm);
    long long accepted = 0, tried = 0, samples = 0;
    const long long total = n_equil + n_sweeps;
    for (long long sweep = 0; sweep < total; ++sweep) {
        for (int m = 0; m < n; ++m) {
            const int i = (int)(uniform(&R) * n);
            double p[3];
            for (int a = 0; a < 3; ++a) {
                double v = x[3 * i + a] + delta * (2.0 * uniform(&R) - 1.0);
                if (v >= L) v -= L;
                if (v < 0) v += L;
                p[a] = v;
            }
            const double e_old = energy_at(&S, i, x + 3 * i);
            const double e_new = energy_at(&S, i, p);
            const double dU = e_new - e_old;
            const int ok = dU <= 0.0 || uniform(&R) < exp(-dU / kT);
            if (sweep >= n_equil) {
                ++tried;
                accepted += ok;
            }
            if (ok) {
                unlink_particle(&S, i);
                for (int a = 0; a < 3; ++a) x[3 * i + a] = p[a];
                insert(&S, i, cell_of(&S, p));
            }
        }
        if (sweep >= n_equil && (sweep - n_equil) % every == 0) {
            accumulate_gr(&S, rmax, nbins, hist);
            ++samples;
        }
    }
    const double pi = 3.14159265358979323846;
    const double dr = rmax / nbins;
    const double pairs = 0.5 * (double)n * (double)(n - 1);
    const double V = L * L * L;
    for (int b = 0; b < nbins; ++b) {
        const double r0 = b * dr, r1 = (b + 1) * dr;
        const double shell = 4.0 / 3.0 * pi * (r1 * r1 * r1 - r0 * r0 * r0);
        gr[b] = samples ? hist[b] / ((double)samples * pairs * shell / V) : 0.0;
    }
    if (acceptance) *acceptance = tried ? (double)accepted / (double)tried : 0.0;
    free(S.head); free(S.next); free(S.prev); free(S.cell); free(hist);
    return 0;
}
