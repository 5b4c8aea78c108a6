/*
 * ORACLE (test infrastructure only) -- plain FP64 transport solve of one
 * (band, direction) system, written for clarity, not speed.
 *
 * Only tests, the smoke check and the benchmark's CPU-baseline leg may load
 * this file's library.  The product path never does.
 *
 * What it computes (Methods, Eq. (4) per mode, and the transport matrix of
 * Eq. (13), A = I/tau + v K_i): the steady per-mode balance over every cell c,
 *
 *   (1/tau + v * sum_{f: a_cf > 0} a_cf) e_c
 *       - v * sum_{f: a_cf < 0} |a_cf| e_up(f)  =  rhs_c,
 *
 * where a_cf = (s . S_cf) / V_c, S_cf = outward area vector of face f of cell
 * c, and e_up(f) is the upwind value: the neighbour's e for an interior face,
 * the prescribed inflow value for a boundary face (first-order upwind finite
 * volume).  A face with a_cf == 0 carries nothing.
 *
 * For first-order upwind the matrix is triangular in the upwind (topological)
 * order of the direction, so the exact solve is a forward substitution in
 * that order.  The order is found with Kahn's algorithm; if the upwind graph
 * has a cycle the function reports it and the caller solves the system with a
 * sparse direct solver instead.
 *
 * Outputs per cell: e_c, and outflux_c = sum_f a_cf e_up(f) (outgoing faces
 * carry e_c), the per-volume net outflow of this system without the factor v,
 * used by the caller for the face-based divergence of the heat flux.
 */
#include <stdint.h>
#include <stdlib.h>

/* returns 0 on success, 1 if the upwind graph of this direction is cyclic,
   2 on allocation failure */
int oracle_sweep_system(int64_t N, int32_t F,
                        const int64_t *nbr,    /* N*F: >=0 neighbour cell, <0: -(1+boundary face index) */
                        const double *S,       /* N*F*3 outward area vectors */
                        const double *V,       /* N cell volumes */
                        const double *s,       /* 3: direction */
                        double v, double inv_tau,
                        const double *rhs,     /* N */
                        const double *inflow,  /* indexed by boundary face index */
                        double *e,             /* N out */
                        double *outflux)       /* N out */
{
    int64_t *indeg = (int64_t *)calloc((size_t)N, sizeof(int64_t));
    int64_t *order = (int64_t *)malloc((size_t)N * sizeof(int64_t));
    double *a = (double *)malloc((size_t)N * (size_t)F * sizeof(double));
    if (!indeg || !order || !a) { free(indeg); free(order); free(a); return 2; }

    /* a_cf for this direction */
    for (int64_t c = 0; c < N; ++c)
        for (int32_t f = 0; f < F; ++f) {
            const double *Sf = S + 3 * (c * F + f);
            a[c * F + f] = (s[0] * Sf[0] + s[1] * Sf[1] + s[2] * Sf[2]) / V[c];
        }

    /* in-degree: number of interior upwind neighbours of each cell */
    for (int64_t c = 0; c < N; ++c)
        for (int32_t f = 0; f < F; ++f)
            if (a[c * F + f] < 0.0 && nbr[c * F + f] >= 0) indeg[c] += 1;

    /* Kahn's algorithm: a cell is ready once all its upwind neighbours are done.
       Downwind neighbours of u are the cells d that see u across a face with
       a_df < 0, i.e. the faces of u with a_uf > 0 that lead to an interior cell. */
    int64_t head = 0, tail = 0;
    for (int64_t c = 0; c < N; ++c)
        if (indeg[c] == 0) order[tail++] = c;
    while (head < tail) {
        int64_t u = order[head++];
        for (int32_t f = 0; f < F; ++f) {
            int64_t d = nbr[u * F + f];
            if (d >= 0 && a[u * F + f] > 0.0) {
                indeg[d] -= 1;
                if (indeg[d] == 0) order[tail++] = d;
            }
        }
    }
    if (tail != N) { free(indeg); free(order); free(a); return 1; }

    /* forward substitution in upwind order */
    for (int64_t k = 0; k < N; ++k) {
        int64_t c = order[k];
        double diag = inv_tau;
        double gain = 0.0;
        for (int32_t f = 0; f < F; ++f) {
            double acf = a[c * F + f];
            if (acf > 0.0) {
                diag += v * acf;
            } else if (acf < 0.0) {
                int64_t n = nbr[c * F + f];
                double up = (n >= 0) ? e[n] : inflow[-(n + 1)];
                gain += v * (-acf) * up;
            }
        }
        e[c] = (rhs[c] + gain) / diag;
    }

    /* net outflow per unit volume (without v) */
    for (int64_t c = 0; c < N; ++c) {
        double sum = 0.0;
        for (int32_t f = 0; f < F; ++f) {
            double acf = a[c * F + f];
            if (acf > 0.0) {
                sum += acf * e[c];
            } else if (acf < 0.0) {
                int64_t n = nbr[c * F + f];
                double up = (n >= 0) ? e[n] : inflow[-(n + 1)];
                sum += acf * up;
            }
        }
        outflux[c] = sum;
    }
    free(indeg); free(order); free(a);
    return 0;
}

/*
 * All (band, direction) systems of one iteration: the systems are independent
 * within an iteration (Methods, Eq. (14)), so they are simply looped over,
 * one OpenMP thread per system.
 *
 * Layouts: rhs[b*N + c]; inflow[(b*D + i)*NBF + bf]; e and outflux
 * [(b*D + i)*N + c].  status[b*D + i] receives the per-system return code.
 */
void oracle_sweep_all(int64_t N, int32_t F, int32_t B, int32_t D, int64_t NBF,
                      const int64_t *nbr, const double *S, const double *V,
                      const double *dirs /* D*3 */, const double *vel /* B */,
                      const double *inv_tau /* B */, const double *rhs,
                      const double *inflow, double *e, double *outflux, int32_t *status)
{
    int64_t nsys = (int64_t)B * D;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < nsys; ++k) {
        int32_t b = (int32_t)(k / D), i = (int32_t)(k % D);
        status[k] = oracle_sweep_system(N, F, nbr, S, V, dirs + 3 * i, vel[b], inv_tau[b],
                                        rhs + (int64_t)b * N, inflow + k * NBF,
                                        e + k * N, outflux + k * N);
    }
}

/*
 * The same with a right-hand side per system, rhs[(b*D + i)*N + c] (the
 * second-order scheme's deferred correction differs between directions).
 */
void oracle_sweep_all_sys(int64_t N, int32_t F, int32_t B, int32_t D, int64_t NBF,
                          const int64_t *nbr, const double *S, const double *V,
                          const double *dirs, const double *vel, const double *inv_tau, const double *rhs,
                          const double *inflow, double *e, double *outflux, int32_t *status)
{
    int64_t nsys = (int64_t)B * D;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < nsys; ++k) {
        int32_t b = (int32_t)(k / D), i = (int32_t)(k % D);
        status[k] = oracle_sweep_system(N, F, nbr, S, V, dirs + 3 * i, vel[b], inv_tau[b],
                                        rhs + k * N, inflow + k * NBF, e + k * N, outflux + k * N);
    }
}

/*
 * Threads of the OpenMP loop above: n > 0 sets them, every call returns the
 * number the next loop will use (the CPU baseline reports it).
 */
#include <omp.h>
int oracle_threads(int n)
{
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
}
