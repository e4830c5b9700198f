/*
 * d3q19_oracle.c -- FP64 reference for the D3Q19 extension of the lattice
 * update (test infrastructure only: the test suite, the smoke check and the
 * CPU baseline of the benchmark use it; the HIP library never does).
 *
 * The paper names the 3-D extension as future work (Section 6); this is the
 * same method with the D3Q19 velocity set:
 *   - Velocities: the 19 vectors c with components in {-1, 0, 1} and
 *     |c|^2 <= 2, ordered by (c_z, c_y, c_x) lexicographically, so that the
 *     rest vector is i = 9 and opposite(i) = 18 - i.  Weights 1/3 (rest),
 *     1/18 (|c| = 1), 1/36 (|c|^2 = 2): the unique weights of this set with
 *     the isotropy of Eq. 2's moments.
 *   - Collision: BGK (Eq. 1) with the incompressible equilibrium of Eq. 2,
 *     feq_i = w_i (rho + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u), u = sum f c, and
 *     the force term 3 w_i (c_i . g).
 *   - Streaming: two-lattice pull (Section 3.3), one step.
 *   - Halfway bounce-back at fluid-solid links and at closed sides.
 *   - Inlet column x = 0 with fixed feq(1, u_in); outlet column x = nx - 1
 *     with zero gradient (a pull from beyond it takes the last column's
 *     value, after the y and z shifts).
 *
 * Layout of this file's arrays: node n = (z ny + y) nx + x; populations
 * f[n * 19 + i] (pull state: post-collision, not yet streamed).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { O3_FLUID = 0, O3_SOLID = 1, O3_INLET = 2, O3_OUTLET = 3 };
enum { O3_PERIODIC = 0, O3_CLOSED = 1, O3_INFLOW_OUTFLOW = 2 };

typedef struct {
    int64_t nx, ny, nz;
    int32_t x_axis, y_axis, z_axis, pad;
    double tau;
    double u_in[3], g[3], u0[3];
} ora3_params;

static int CX[19], CY[19], CZ[19];
static double W[19];
static int ready = 0;

/* The velocity set and its weights, generated from their definition. */
static void setup(void)
{
    if (ready) return;
    int i = 0;
    for (int z = -1; z <= 1; ++z)
        for (int y = -1; y <= 1; ++y)
            for (int x = -1; x <= 1; ++x) {
                const int c2 = x * x + y * y + z * z;
                if (c2 > 2) continue;
                CX[i] = x;
                CY[i] = y;
                CZ[i] = z;
                W[i] = c2 == 0 ? 1.0 / 3.0 : (c2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
                ++i;
            }
    ready = 1;
}

void ora3_constants(int* cx, int* cy, int* cz, double* w)
{
    setup();
    for (int i = 0; i < 19; ++i) {
        cx[i] = CX[i];
        cy[i] = CY[i];
        cz[i] = CZ[i];
        w[i] = W[i];
    }
}

static void equilibrium(double rho, const double u[3], double* feq)
{
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < 19; ++i) {
        const double cu = CX[i] * u[0] + CY[i] * u[1] + CZ[i] * u[2];
        feq[i] = W[i] * (rho + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
    }
}

void ora3_equilibrium(double rho, double ux, double uy, double uz, double* feq)
{
    setup();
    const double u[3] = {ux, uy, uz};
    equilibrium(rho, u, feq);
}

static int updated(uint8_t t) { return t == O3_FLUID || t == O3_OUTLET; }

int ora3_node_types(const ora3_params* p, const uint8_t* flags, uint8_t* types)
{
    setup();
    const int64_t N = p->nx * p->ny * p->nz;
    for (int64_t n = 0; n < N; ++n) {
        const int64_t x = n % p->nx;
        uint8_t t = O3_FLUID;
        if (flags[n]) t = O3_SOLID;
        else if (p->x_axis == O3_INFLOW_OUTFLOW && x == 0) t = O3_INLET;
        else if (p->x_axis == O3_INFLOW_OUTFLOW && x == p->nx - 1) t = O3_OUTLET;
        types[n] = t;
    }
    return 0;
}

int ora3_init_state(const ora3_params* p, const uint8_t* types, double* f)
{
    setup();
    double e0[19], ein[19];
    equilibrium(1.0, p->u0, e0);
    equilibrium(1.0, p->u_in, ein);
    const int64_t N = p->nx * p->ny * p->nz;
    for (int64_t n = 0; n < N; ++n)
        for (int i = 0; i < 19; ++i)
            f[n * 19 + i] = updated(types[n]) ? e0[i] : (types[n] == O3_INLET ? ein[i] : 0.0);
    return 0;
}

/* Source coordinate along one axis after its rule: 1 inside, 0 outside a
 * closed side (solid).  The inflow/outflow rule clamps past the outlet. */
static int axis_rule(int kind, int64_t n, int64_t* s)
{
    if (*s >= 0 && *s < n) return 1;
    if (kind == O3_PERIODIC) {
        *s = *s < 0 ? *s + n : *s - n;
        return 1;
    }
    if (kind == O3_INFLOW_OUTFLOW && *s >= n) {
        *s = n - 1;
        return 1;
    }
    return 0;
}

/* Incoming value of direction i at node (x, y, z). */
static double pull_one(const ora3_params* p, const uint8_t* types, const double* f, const double* ein,
                       int64_t x, int64_t y, int64_t z, int i)
{
    int64_t sx = x - CX[i], sy = y - CY[i], sz = z - CZ[i];
    const int64_t self = (z * p->ny + y) * p->nx + x;
    int inside = axis_rule(p->y_axis, p->ny, &sy) && axis_rule(p->z_axis, p->nz, &sz) &&
                 axis_rule(p->x_axis, p->nx, &sx);
    if (inside) {
        const int64_t s = (sz * p->ny + sy) * p->nx + sx;
        if (types[s] == O3_INLET) return ein[i];
        if (types[s] != O3_SOLID) return f[s * 19 + i];
    }
    return f[self * 19 + (18 - i)]; /* halfway bounce-back */
}

static void gather_node(const ora3_params* p, const uint8_t* types, const double* f, const double* ein,
                        int64_t x, int64_t y, int64_t z, double* fin)
{
    for (int i = 0; i < 19; ++i) fin[i] = pull_one(p, types, f, ein, x, y, z, i);
}

int ora3_gather(const ora3_params* p, const uint8_t* types, const double* f, double* fin)
{
    setup();
    double ein[19];
    equilibrium(1.0, p->u_in, ein);
    const int64_t N = p->nx * p->ny * p->nz;
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        const int64_t x = n % p->nx, y = (n / p->nx) % p->ny, z = n / (p->nx * p->ny);
        double v[19];
        if (updated(types[n]))
            gather_node(p, types, f, ein, x, y, z, v);
        else
            for (int i = 0; i < 19; ++i) v[i] = types[n] == O3_INLET ? ein[i] : 0.0;
        memcpy(fin + n * 19, v, sizeof(v));
    }
    return 0;
}

static void step(const ora3_params* p, const uint8_t* types, const double* f, double* fnew)
{
    double ein[19];
    equilibrium(1.0, p->u_in, ein);
    const int64_t N = p->nx * p->ny * p->nz;
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        if (!updated(types[n])) {
            memcpy(fnew + n * 19, f + n * 19, 19 * sizeof(double));
            continue;
        }
        const int64_t x = n % p->nx, y = (n / p->nx) % p->ny, z = n / (p->nx * p->ny);
        double fin[19], feq[19], u[3] = {0, 0, 0}, rho = 0.0;
        gather_node(p, types, f, ein, x, y, z, fin);
        for (int i = 0; i < 19; ++i) {
            rho += fin[i];
            u[0] += fin[i] * CX[i];
            u[1] += fin[i] * CY[i];
            u[2] += fin[i] * CZ[i];
        }
        equilibrium(rho, u, feq);
        for (int i = 0; i < 19; ++i) {
            const double force = 3.0 * W[i] * (CX[i] * p->g[0] + CY[i] * p->g[1] + CZ[i] * p->g[2]);
            fnew[n * 19 + i] = fin[i] - (fin[i] - feq[i]) / p->tau + force;
        }
    }
}

int ora3_run(const ora3_params* p, const uint8_t* types, double* f, double* tmp, int64_t steps)
{
    setup();
    double* a = f;
    double* b = tmp;
    for (int64_t s = 0; s < steps; ++s) {
        step(p, types, a, b);
        double* t = a;
        a = b;
        b = t;
    }
    if (a != f) memcpy(f, a, (size_t)(p->nx * p->ny * p->nz * 19) * sizeof(double));
    return 0;
}

/* rho and u (+ g/2) from the incoming values; inlet (1, u_in); solid 0. */
int ora3_readout(const ora3_params* p, const uint8_t* types, const double* f, double* rho, double* u)
{
    setup();
    double ein[19];
    equilibrium(1.0, p->u_in, ein);
    const int64_t N = p->nx * p->ny * p->nz;
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        const int64_t x = n % p->nx, y = (n / p->nx) % p->ny, z = n / (p->nx * p->ny);
        double r = 0.0, j[3] = {0, 0, 0};
        if (updated(types[n])) {
            double v[19];
            gather_node(p, types, f, ein, x, y, z, v);
            for (int i = 0; i < 19; ++i) {
                r += v[i];
                j[0] += v[i] * CX[i];
                j[1] += v[i] * CY[i];
                j[2] += v[i] * CZ[i];
            }
            for (int a = 0; a < 3; ++a) j[a] += 0.5 * p->g[a];
        } else if (types[n] == O3_INLET) {
            r = 1.0;
            for (int a = 0; a < 3; ++a) j[a] = p->u_in[a];
        }
        rho[n] = r;
        for (int a = 0; a < 3; ++a) u[a * N + n] = j[a];
    }
    return 0;
}
