/*
 * lbm_oracle.c -- plain FP64 CPU reference of the D2Q9I BGK lattice update.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the HIP path is
 * checked against; it shares no code, header, table or constant with the
 * library under paper_2607_20650_amd/ and is never linked into it.  Only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark load
 * it.
 *
 * What it computes (paper, Section 3.1, Eq. 1-2, and Section 3.3):
 *   - D2Q9 velocity set in the order of Fig. 2 (b):  SW S SE W 0 E NW N NE,
 *     y growing upwards; weights of Eq. 2 (4/9 rest, 1/9 axis, 1/36 diagonal).
 *   - Incompressible equilibrium of Eq. 2 (D2Q9I):
 *         feq_i = w_i [rho + 3 v.c_i + 9/2 (v.c_i)^2 - 3/2 v.v],
 *     with v = sum_i f_i c_i (no division by rho).
 *   - BGK relaxation of Eq. 1 with time step 1:
 *         f_i(r + c_i, t + 1) = f_i - (f_i - feq_i) / tau.
 *   - Two lattices and one-step pull streaming (the paper's basic
 *     two-lattice approach): every node pulls its incoming values, collides,
 *     and writes to the second lattice; the lattices then swap roles.
 *   - Halfway bounce-back at fluid-solid links (Section 3.1, last
 *     paragraph): a value that would come from a solid node is replaced by the
 *     node's own post-collision value of the opposite direction.  Optionally
 *     (fullway = 1) full-way bounce-back instead: solid nodes hold populations
 *     (initially at rest), take in what streams into them like any node and,
 *     in place of collision, reverse every direction; a fluid node pulls from a
 *     solid node like from any other.  Closed sides stay halfway.
 *   - Inlet: equilibrium feq(rho_in, u_in) (Section 3.1): Dirichlet, rho_in = 1,
 *     or Neumann, rho_in = the density of the adjacent node of column 1 in the
 *     previous update (the sum of its post-collision values held in the state,
 *     collision and force conserving mass).  Outlet: zero gradient (a pull across the
 *     last column takes the value from the last column), or the pressure
 *     outlet of Zou and He that Section 3.1 adapts: at an outlet node the
 *     three incoming values with c_x = -1 are rebuilt from the six others so
 *     that the node's incoming density is 1 and its tangential momentum zero,
 *     the normal non-equilibrium parts bouncing back (the incompressible
 *     model's momentum j in place of rho u).
 *   - Body force (an addition, not in the paper): after relaxation every
 *     updated node adds 3 w_i (c_i . g); reported velocity is j + g/2.
 *
 * State convention: f holds, for every node, the post-collision values f*_i
 * that have not yet streamed ("pull state"), laid out f[(y*nx + x)*9 + i].
 * Readout at time t gathers the incoming values exactly as a step would and
 * takes their moments.
 *
 * Parallelism: OpenMP over rows (plain static schedule), nothing else.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Node types after derivation from the user flags. */
enum { ORA_FLUID = 0, ORA_SOLID = 1, ORA_INLET = 2, ORA_OUTLET = 3 };
/* Axis kinds. */
enum { ORA_PERIODIC = 0, ORA_CLOSED = 1, ORA_INFLOW_OUTFLOW = 2, ORA_INFLOW_PRESSURE = 3,
       ORA_NEUMANN_OUTFLOW = 4, ORA_NEUMANN_PRESSURE = 5 };

/* Inlet at column 0 and outlet at column nx-1 on the x axis. */
static int inout(int axis) { return axis >= ORA_INFLOW_OUTFLOW && axis <= ORA_NEUMANN_PRESSURE; }
/* Outlet kind: pressure (Zou-He) or zero gradient. */
static int pressure_outlet(int axis) { return axis == ORA_INFLOW_PRESSURE || axis == ORA_NEUMANN_PRESSURE; }
/* Inlet density kind: Neumann (copied from column 1) or Dirichlet (1). */
static int neumann_inlet(int axis) { return axis == ORA_NEUMANN_OUTFLOW || axis == ORA_NEUMANN_PRESSURE; }

/* Fig. 2 (b): SW, S, SE, W, rest, E, NW, N, NE. */
static const int CX[9] = {-1, 0, 1, -1, 0, 1, -1, 0, 1};
static const int CY[9] = {-1, -1, -1, 0, 0, 0, 1, 1, 1};
static const int OPP[9] = {8, 7, 6, 5, 4, 3, 2, 1, 0};
/* Eq. 2: w4 = 4/9; w1, w3, w5, w7 = 1/9; w0, w2, w6, w8 = 1/36. */
static const double W[9] = {1.0 / 36, 1.0 / 9, 1.0 / 36, 1.0 / 9, 4.0 / 9,
                            1.0 / 9, 1.0 / 36, 1.0 / 9, 1.0 / 36};

typedef struct {
    int64_t nx, ny;
    int32_t x_axis, y_axis; /* ORA_PERIODIC / ORA_CLOSED / ORA_INFLOW_OUTFLOW (x only) /
                               ORA_INFLOW_PRESSURE (x only) */
    double tau;
    double u_in[2];
    double g[2];
    double u0[2];
    int32_t fullway; /* 1: full-way bounce-back at solid nodes, 0: halfway */
    int32_t pad;
} ora_params;

int ora_abi_version(void) { return 1; }

void ora_constants(int* cx, int* cy, int* opp, double* w)
{
    for (int i = 0; i < 9; ++i) {
        cx[i] = CX[i];
        cy[i] = CY[i];
        opp[i] = OPP[i];
        w[i] = W[i];
    }
}

/* Eq. 2 for density rho and velocity (vx, vy). */
static void equilibrium(double rho, double vx, double vy, double feq[9])
{
    double vv = vx * vx + vy * vy;
    for (int i = 0; i < 9; ++i) {
        double vc = vx * CX[i] + vy * CY[i];
        feq[i] = W[i] * (rho + 3.0 * vc + 4.5 * vc * vc - 1.5 * vv);
    }
}

void ora_equilibrium(double rho, double vx, double vy, double* feq) { equilibrium(rho, vx, vy, feq); }

/* Node types: solid where the user says so; with an inflow/outflow x axis the
 * first column is inlet and the last column outlet (solid wins). */
int ora_node_types(const ora_params* p, const uint8_t* flags, uint8_t* types)
{
    for (int64_t y = 0; y < p->ny; ++y)
        for (int64_t x = 0; x < p->nx; ++x) {
            int64_t n = y * p->nx + x;
            uint8_t t = ORA_FLUID;
            if (flags[n] != 0)
                t = ORA_SOLID;
            else if (inout(p->x_axis) && x == 0)
                t = ORA_INLET;
            else if (inout(p->x_axis) && x == p->nx - 1)
                t = ORA_OUTLET;
            types[n] = t;
        }
    return 0;
}

/* Initial pull state: fluid and outlet feq(1, u0), inlet feq(1, u_in), solid 0. */
int ora_init_state(const ora_params* p, const uint8_t* types, double* f)
{
    double e0[9], ein[9];
    equilibrium(1.0, p->u0[0], p->u0[1], e0);
    equilibrium(1.0, p->u_in[0], p->u_in[1], ein);
    int64_t N = p->nx * p->ny;
    for (int64_t n = 0; n < N; ++n)
        for (int i = 0; i < 9; ++i) {
            double v = 0.0;
            if (types[n] == ORA_FLUID || types[n] == ORA_OUTLET) v = e0[i];
            if (types[n] == ORA_INLET) v = ein[i];
            if (types[n] == ORA_SOLID && p->fullway) v = W[i]; /* at rest */
            f[n * 9 + i] = v;
        }
    return 0;
}

/* Incoming value of direction i at node (x, y): the post-collision value that
 * streams in from (x - c_i, y - c_i), with the boundary rules applied. */
static double pull_one(const ora_params* p, const uint8_t* types, const double* f,
                       const double* ein, int64_t x, int64_t y, int i)
{
    int64_t sx = x - CX[i];
    int64_t sy = y - CY[i];
    int solid = 0;
    if (sy < 0 || sy >= p->ny) {
        if (p->y_axis == ORA_PERIODIC)
            sy = (sy + p->ny) % p->ny;
        else
            solid = 1; /* closed: outside the box behaves like a wall */
    }
    if (sx < 0 || sx >= p->nx) {
        if (p->x_axis == ORA_PERIODIC)
            sx = (sx + p->nx) % p->nx;
        else if (inout(p->x_axis) && sx >= p->nx)
            sx = p->nx - 1; /* zero gradient across the outlet */
        else
            solid = 1;
    }
    if (!solid) {
        uint8_t t = types[sy * p->nx + sx];
        if (t == ORA_SOLID && !p->fullway) solid = 1;
        else if (t == ORA_INLET) return ein[sy * 9 + i];
        else return f[(sy * p->nx + sx) * 9 + i];
    }
    /* halfway bounce-back */
    return f[(y * p->nx + x) * 9 + OPP[i]];
}

/* Inlet equilibrium of every row, ein[y * 9 + i] = feq_i(rho_in(y), u_in), from
 * the state f: rho_in = 1 (Dirichlet) or the sum of the post-collision values
 * of node (1, y) (Neumann; 1 where that node is not updated).  Caller frees. */
static double* inlet_rows(const ora_params* p, const uint8_t* types, const double* f)
{
    double* ein = (double*)malloc((size_t)p->ny * 9 * sizeof(double));
    for (int64_t y = 0; y < p->ny; ++y) {
        double rho = 1.0;
        if (neumann_inlet(p->x_axis) && p->nx > 1) {
            const int64_t n = y * p->nx + 1;
            if (types[n] == ORA_FLUID || types[n] == ORA_OUTLET) {
                rho = 0.0;
                for (int i = 0; i < 9; ++i) rho += f[n * 9 + i];
            }
        }
        equilibrium(rho, p->u_in[0], p->u_in[1], ein + y * 9);
    }
    return ein;
}

/* All incoming values of an updated node (x, y).  With the pressure outlet,
 * an outlet node's values arriving from beyond the last column (c_x = -1:
 * directions 0, 3, 6) are replaced: with K the sum of the three c_x = 0 values
 * plus twice the three c_x = +1 values, density 1 requires j_x = K - 1;
 * bouncing back the non-equilibrium part of the normal direction gives
 * f_3 = f_5 - 2 j_x / 3, and zero tangential momentum splits the rest between
 * the two diagonals. */
static void gather_node(const ora_params* p, const uint8_t* types, const double* f, const double* ein,
                        int64_t x, int64_t y, double fin[9])
{
    for (int i = 0; i < 9; ++i) fin[i] = pull_one(p, types, f, ein, x, y, i);
    if (pressure_outlet(p->x_axis) && x == p->nx - 1) {
        const double K = fin[1] + fin[4] + fin[7] + 2.0 * (fin[2] + fin[5] + fin[8]);
        const double jx = K - 1.0;
        fin[3] = fin[5] - 2.0 * jx / 3.0;
        fin[6] = fin[2] + 0.5 * (fin[1] - fin[7]) - jx / 6.0;
        fin[0] = fin[8] - 0.5 * (fin[1] - fin[7]) - jx / 6.0;
    }
}

int ora_gather(const ora_params* p, const uint8_t* types, const double* f, double* fin)
{
    double* ein = inlet_rows(p, types, f);
#pragma omp parallel for schedule(static)
    for (int64_t y = 0; y < p->ny; ++y)
        for (int64_t x = 0; x < p->nx; ++x) {
            int64_t n = y * p->nx + x;
            double v[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
            if (types[n] == ORA_FLUID || types[n] == ORA_OUTLET)
                gather_node(p, types, f, ein, x, y, v);
            else if (types[n] == ORA_INLET)
                for (int i = 0; i < 9; ++i) v[i] = ein[y * 9 + i];
            for (int i = 0; i < 9; ++i) fin[n * 9 + i] = v[i];
        }
    free(ein);
    return 0;
}

/* One lattice update: fnew = collide(pull(f)) on fluid and outlet nodes;
 * inlet and solid nodes keep their (unused) values. */
static void step(const ora_params* p, const uint8_t* types, const double* f, double* fnew)
{
    double* ein = inlet_rows(p, types, f);
    const double tau = p->tau;
#pragma omp parallel for schedule(static)
    for (int64_t y = 0; y < p->ny; ++y)
        for (int64_t x = 0; x < p->nx; ++x) {
            int64_t n = y * p->nx + x;
            if (types[n] == ORA_SOLID && p->fullway) {
                /* full-way bounce-back: a solid node takes in what streams
                 * into it and sends it back the way it came, one update later */
                double fin[9];
                for (int i = 0; i < 9; ++i) fin[i] = pull_one(p, types, f, ein, x, y, i);
                for (int i = 0; i < 9; ++i) fnew[n * 9 + i] = fin[OPP[i]];
                continue;
            }
            if (types[n] != ORA_FLUID && types[n] != ORA_OUTLET) {
                for (int i = 0; i < 9; ++i) fnew[n * 9 + i] = f[n * 9 + i];
                continue;
            }
            double fin[9];
            gather_node(p, types, f, ein, x, y, fin);
            double rho = 0.0, vx = 0.0, vy = 0.0;
            for (int i = 0; i < 9; ++i) {
                rho += fin[i];
                vx += fin[i] * CX[i];
                vy += fin[i] * CY[i];
            }
            double feq[9];
            equilibrium(rho, vx, vy, feq);
            for (int i = 0; i < 9; ++i) {
                double force = 3.0 * W[i] * (CX[i] * p->g[0] + CY[i] * p->g[1]);
                fnew[n * 9 + i] = fin[i] - (fin[i] - feq[i]) / tau + force;
            }
        }
    free(ein);
}

/* Advance `steps` updates.  f (in/out) holds the pull state; tmp is scratch
 * of the same size.  Returns 0. */
int ora_run(const ora_params* p, const uint8_t* types, double* f, double* tmp, int64_t steps)
{
    int64_t N9 = p->nx * p->ny * 9;
    double* a = f;
    double* b = tmp;
    for (int64_t s = 0; s < steps; ++s) {
        step(p, types, a, b);
        double* t = a;
        a = b;
        b = t;
    }
    if (a != f) memcpy(f, a, (size_t)N9 * sizeof(double));
    return 0;
}

/* Macroscopic readout at the current time: rho = sum fin, u = sum fin c + g/2
 * on fluid/outlet nodes; inlet (rho_in, u_in); solid (0, 0). */
int ora_readout(const ora_params* p, const uint8_t* types, const double* f, double* rho, double* ux,
                double* uy)
{
    double* ein = inlet_rows(p, types, f);
#pragma omp parallel for schedule(static)
    for (int64_t y = 0; y < p->ny; ++y)
        for (int64_t x = 0; x < p->nx; ++x) {
            int64_t n = y * p->nx + x;
            double r = 0.0, jx = 0.0, jy = 0.0;
            if (types[n] == ORA_FLUID || types[n] == ORA_OUTLET) {
                double v[9];
                gather_node(p, types, f, ein, x, y, v);
                for (int i = 0; i < 9; ++i) {
                    r += v[i];
                    jx += v[i] * CX[i];
                    jy += v[i] * CY[i];
                }
                jx += 0.5 * p->g[0];
                jy += 0.5 * p->g[1];
            } else if (types[n] == ORA_INLET) {
                for (int i = 0; i < 9; ++i) r += ein[y * 9 + i];
                jx = p->u_in[0];
                jy = p->u_in[1];
            }
            rho[n] = r;
            ux[n] = jx;
            uy[n] = jy;
        }
    free(ein);
    return 0;
}

int ora_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void ora_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
