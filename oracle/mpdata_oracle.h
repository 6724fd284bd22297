/*
 * mpdata_oracle.h -- interface of the FP64 CPU oracle of one MPDATA step.
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
 * baseline of the benchmark.  Shares no code with the HIP library.
 */
#ifndef MPDATA_ORACLE_H
#define MPDATA_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_BC_PERIODIC = 0, ORC_BC_OPEN = 1 };
enum { ORC_MAX_IORD = 16 };

typedef struct {
    int nx, ny, nz; /* cells along x (fastest), y, z */
    int bc;         /* ORC_BC_PERIODIC or ORC_BC_OPEN */
    int iord;       /* 1: donor cell only; k > 1: k - 1 corrective passes */
    int nonos;      /* 1: non-oscillatory limiter on */
    int vsign;      /* 1: fields of variable sign -- |psi1| in the ratios A, B */
    int div;        /* 1: divergent-flow term in the pseudo-velocity */
    double eps;     /* regulariser of ratio denominators */
} orc_params;

/* Optional stage outputs of one step (any pointer may be NULL): psi1 is the
 * first-order result, the others belong to the last corrective pass. */
typedef struct {
    double *psi1;               /* nx*ny*nz */
    double *v1, *v2, *v3;       /* unlimited pseudo-velocities, face arrays */
    double *mx, *mn;            /* limiter bounds */
    double *beta_up, *beta_dn;  /* limiter factors */
} orc_stages;

/* 0 if the parameters are valid, -1 otherwise. */
int orc_check(const orc_params *p);

/* One step psi -> out.  Returns 0, -1 on bad parameters, -2 on allocation
 * failure.  psi and out must not alias. */
int orc_step(const orc_params *p, const double *psi, const double *u1,
             const double *u2, const double *u3, const double *h, double *out,
             orc_stages *stages);

/* One step with Courant numbers that change in time: u1..u3 at the start of
 * the step (level n), w1..w3 at its end (level n+1).  The first corrective
 * pass adds (w - u)/2 to the pseudo-velocity of every face (zero on the
 * boundary-normal faces of an open domain).  w1..w3 all NULL: orc_step. */
int orc_step_tv(const orc_params *p, const double *psi, const double *u1,
                const double *u2, const double *u3, const double *w1,
                const double *w2, const double *w3, const double *h, double *out,
                orc_stages *stages);

/* nsteps steps in place on psi. */
int orc_run(const orc_params *p, double *psi, const double *u1, const double *u2,
            const double *u3, const double *h, int nsteps);

/* Compensated sum of h[i]*psi[i] (Ogita-Rump-Oishi Dot2). */
double orc_mass(long n, const double *h, const double *psi);

/* Net inflow of the first-order pass through the faces of an open domain. */
double orc_open_inflow(const orc_params *p, const double *psi, const double *u1,
                       const double *u2, const double *u3);

/* Threads used by the stage loops, and setting them (n >= 1; returns the
 * number now in effect).  No result depends on the thread count. */
int orc_threads(void);
int orc_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
