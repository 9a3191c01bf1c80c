/*
 * FP64 reference implementation of the Yee FDTD path used by the S-parameter
 * workflow (paper Sec. II-A).  TEST INFRASTRUCTURE ONLY: it exists so that the
 * GPU library can be checked against a plain, slow, obviously correct CPU
 * computation.  Nothing in the product path may link or call it.
 *
 * What it computes, in the order of one time step n -> n+1:
 *   1. H^{n+1/2} from H^{n-1/2} and curl E^n (Yee 1966 staggering, the grid
 *      cited in Sec. II-A), with convolutional-PML auxiliary terms inside
 *      the absorbing layers (the paper uses a PML on every face except the
 *      ground, Sec. II-A; the convolutional form of Roden and Gedney and its
 *      polynomial grading follow Taflove and Hagness, 3rd ed., ch. 7).
 *   2. E^{n+1} = Ca E^n + Cb curl H^{n+1/2} with per-edge Ca, Cb from the
 *      averaged permittivity and conductivity; PEC edges (metal, the ground)
 *      keep E = 0 (Sec. II-A, Sec. II-B).
 *   3. Soft source: E += s(t_{n+1}) on the excitation nodes (eq. 3 and the
 *      soft-source remark that follows it; the paper drives Ez).
 *   4. Port voltage (surface integral of Ez over the plane between the
 *      conductors divided by the strip width) and port current (closed line
 *      integral of H around the strip), eq. 4; point probes.
 *   5. Running DFT of every probe signal at its true sample time (the DFT of
 *      the V and I histories in Sec. II-A).
 * All arithmetic is FP64.  Loops are plain triple loops over the staggered
 * index ranges; OpenMP splits the outermost (z) loop only.
 *
 * Parity notes: the discrete energy invariant, the exact single-mode Yee
 * evolution, cavity resonances, the parallel-plate impedance and the source
 * spectrum pin this file (see the oracle tests).  The edge averaging of the
 * permittivity at material interfaces, a reading the paper leaves open, is
 * pinned by modes in 1-cell alternating layers.  The absorbing-layer
 * defaults, another such reading, are pinned only through the absorption
 * of each axis, not value by value: parity unpinned there.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define FACE_PEC 0
#define FACE_CPML 1
#define FACE_PMC 2

typedef struct {
    int32_t nx, ny, nz;
    double dx, dy, dz;
    double courant;            /* fraction of the 3-D stability limit */
    int32_t normalized;        /* 1: c = eps0 = mu0 = 1 */
    int32_t nmat;
    const double *mat_eps;
    const double *mat_sigma;
    const int32_t *mat_pec;
    const uint8_t *cells;      /* [nz][ny][nx] */
    int32_t face[6];           /* x-, x+, y-, y+, z-, z+ */
    int32_t pml_cells[6];
    double pml_m, pml_sigma_max, pml_kappa_max, pml_alpha_max;
    int32_t src_kind;          /* 0 none, 1 Gaussian in steps, 2 Gaussian sine, 3 differential Gaussian,
                                  4 sampled */
    int32_t src_comp;          /* E component driven (0 Ex, 1 Ey, 2 Ez) */
    int32_t src_box[6];        /* its nodes i0,i1,j0,j1,k0,k1 inclusive */
    double src_t0, src_width, src_fc, src_bw, src_amp;
    int32_t nport;
    const int32_t *ports;      /* 6 per port: i, dir, y0, y1, z0, z1 */
    int32_t npoint;
    const int32_t *points;     /* 4 per point: comp, i, j, k */
    int32_t nf;
    const double *freqs;
    int64_t src_nsamp;         /* sampled source: values for levels 1..src_nsamp */
    const double *src_samples;
} or_problem;

/* Every array is allocated by the caller.  Field and auxiliary arrays are
 * (nx+1)(ny+1)(nz+1) doubles indexed i + (nx+1)(j + (ny+1)k); a component
 * only uses its own staggered index range, the rest stays zero. */
typedef struct {
    double *e[3], *h[3];
    /* PML auxiliaries, by component and derivative axis:
     * hxy hxz hyz hyx hzx hzy exy exz eyz eyx ezx ezy */
    double *psi[12];
    double *ca[3], *cb[3];
    /* 1-D profiles per axis: b, c, 1/kappa at integer (E) and half (H)
     * positions, and an in-layer flag */
    double *bE[3], *cE[3], *ikE[3], *bH[3], *cH[3], *ikH[3];
    int32_t *inE[3], *inH[3];
    double *acc;               /* [probe][2][nf][2] running DFT (re, im) */
    double *hist;              /* [probe][2][hist_len] or NULL */
    int64_t hist_len;
    double *energy;            /* [hist_len] or NULL: W^n for n = step index before the step */
    int64_t step;              /* completed steps */
} or_state;

static double c0_of(const or_problem *p) { return p->normalized ? 1.0 : 299792458.0; }
static double mu0_of(const or_problem *p) { return p->normalized ? 1.0 : 4.0e-7 * M_PI; }
static double eps0_of(const or_problem *p)
{
    double c = c0_of(p);
    return 1.0 / (mu0_of(p) * c * c);
}

/* Time step: the Courant fraction of the 3-D stability limit of the Yee grid. */
double or_dt(const or_problem *p)
{
    double s = 1.0 / (p->dx * p->dx) + 1.0 / (p->dy * p->dy) + 1.0 / (p->dz * p->dz);
    return p->courant / (c0_of(p) * sqrt(s));
}

static size_t idx(const or_problem *p, int i, int j, int k)
{
    return (size_t)i + (size_t)(p->nx + 1) * ((size_t)j + (size_t)(p->ny + 1) * (size_t)k);
}

static int cell_mat(const or_problem *p, int i, int j, int k)
{
    return p->cells[(size_t)i + (size_t)p->nx * ((size_t)j + (size_t)p->ny * (size_t)k)];
}

/* Per-edge update coefficients.  comp 0/1/2 = Ex/Ey/Ez.  The edge is PEC if it
 * lies tangentially on a PEC or absorbing-layer face (the layers are backed by
 * PEC) or if any cell sharing it is PEC; otherwise eps and sigma are the
 * arithmetic means over the cells sharing the edge. */
static void edge_coef(const or_problem *p, double dt, int comp, int i, int j, int k,
                      double *ca, double *cb)
{
    int n[3] = {p->nx, p->ny, p->nz};
    int pos[3] = {i, j, k};
    int a;
    /* tangential on a domain face? the edge is along axis comp, so it is
     * tangential to faces normal to the two other axes */
    for (a = 0; a < 3; ++a) {
        if (a == comp) continue;
        if (pos[a] == 0 && p->face[2 * a] != FACE_PMC) { *ca = 0; *cb = 0; return; }
        if (pos[a] == n[a] && p->face[2 * a + 1] != FACE_PMC) { *ca = 0; *cb = 0; return; }
    }
    /* cells sharing the edge: along comp the cell index equals the edge's,
     * along each other axis it is pos-1 or pos (when inside the grid) */
    int lo[3], hi[3];
    for (a = 0; a < 3; ++a) {
        if (a == comp) { lo[a] = pos[a]; hi[a] = pos[a]; }
        else {
            lo[a] = pos[a] - 1 < 0 ? 0 : pos[a] - 1;
            hi[a] = pos[a] > n[a] - 1 ? n[a] - 1 : pos[a];
        }
    }
    double se = 0, ss = 0;
    int cnt = 0, ci, cj, ck;
    for (ck = lo[2]; ck <= hi[2]; ++ck)
        for (cj = lo[1]; cj <= hi[1]; ++cj)
            for (ci = lo[0]; ci <= hi[0]; ++ci) {
                int m = cell_mat(p, ci, cj, ck);
                if (p->mat_pec[m]) { *ca = 0; *cb = 0; return; }
                se += p->mat_eps[m];
                ss += p->mat_sigma[m];
                ++cnt;
            }
    double eps = eps0_of(p) * se / cnt;
    double sig = ss / cnt;
    double loss = sig * dt / (2.0 * eps);
    *ca = (1.0 - loss) / (1.0 + loss);
    *cb = (dt / eps) / (1.0 + loss);
}

/* Convolutional-PML profile value at a coordinate pos (in cells) on axis a. */
static void pml_point(const or_problem *p, double dt, int a, double pos,
                      double *b, double *c, double *ik, int32_t *in)
{
    int n[3] = {p->nx, p->ny, p->nz};
    double dl[3] = {p->dx, p->dy, p->dz};
    int Llo = p->face[2 * a] == FACE_CPML ? p->pml_cells[2 * a] : 0;
    int Lhi = p->face[2 * a + 1] == FACE_CPML ? p->pml_cells[2 * a + 1] : 0;
    double rho = 0, d = 1;
    if (Llo > 0 && pos < Llo) { rho = Llo - pos; d = Llo; }
    if (Lhi > 0 && pos > n[a] - Lhi) { rho = pos - (n[a] - Lhi); d = Lhi; }
    *b = 1.0; *c = 0.0; *ik = 1.0; *in = 0;
    if (rho <= 0) return;
    double eps0 = eps0_of(p);
    double eta0 = mu0_of(p) * c0_of(p);
    double m = p->pml_m;
    double smax = p->pml_sigma_max > 0 ? p->pml_sigma_max : 0.8 * (m + 1.0) / (eta0 * dl[a]);
    double x = rho / d;
    double sig = smax * pow(x, m);
    double kap = 1.0 + (p->pml_kappa_max - 1.0) * pow(x, m);
    double alp = p->pml_alpha_max * (1.0 - x);
    *b = exp(-(sig / kap + alp) * dt / eps0);
    *c = (sig + kap * alp) > 0 ? sig * (*b - 1.0) / (kap * (sig + kap * alp)) : 0.0;
    *ik = 1.0 / kap;
    *in = 1;
}

int or_setup(const or_problem *p, or_state *s)
{
    double dt = or_dt(p);
    int n[3] = {p->nx, p->ny, p->nz};
    int a, i, j, k, comp;
    for (a = 0; a < 3; ++a) {
        for (i = 0; i <= n[a]; ++i)
            pml_point(p, dt, a, (double)i, &s->bE[a][i], &s->cE[a][i], &s->ikE[a][i], &s->inE[a][i]);
        for (i = 0; i < n[a]; ++i)
            pml_point(p, dt, a, i + 0.5, &s->bH[a][i], &s->cH[a][i], &s->ikH[a][i], &s->inH[a][i]);
    }
    for (comp = 0; comp < 3; ++comp) {
        int ni = p->nx - (comp == 0), nj = p->ny - (comp == 1), nk = p->nz - (comp == 2);
#pragma omp parallel for private(i, j) schedule(static)
        for (k = 0; k <= nk; ++k)
            for (j = 0; j <= nj; ++j)
                for (i = 0; i <= ni; ++i) {
                    size_t id = idx(p, i, j, k);
                    edge_coef(p, dt, comp, i, j, k, &s->ca[comp][id], &s->cb[comp][id]);
                }
    }
    return 0;
}

/* Tangential H just outside a face: the mirror image (with a sign flip) on a
 * magnetic wall, zero elsewhere (there the E edge it feeds is PEC anyway). */
static double hval(const or_problem *p, const or_state *s, int comp, int i, int j, int k)
{
    int n[3] = {p->nx, p->ny, p->nz};
    int pos[3] = {i, j, k};
    int a;
    for (a = 0; a < 3; ++a) {
        if (pos[a] < 0) {
            if (p->face[2 * a] != FACE_PMC) return 0.0;
            pos[a] = 0;
            return -s->h[comp][idx(p, pos[0], pos[1], pos[2])];
        }
        /* the last stored half-cell index along a (for the component
         * staggered there) is n-1; index n lies outside */
        if (pos[a] >= n[a] && a != comp) {
            if (p->face[2 * a + 1] != FACE_PMC) return 0.0;
            pos[a] = n[a] - 1;
            return -s->h[comp][idx(p, pos[0], pos[1], pos[2])];
        }
    }
    return s->h[comp][idx(p, i, j, k)];
}

static double waveform(const or_problem *p, double dt, int64_t level)
{
    double t = level * dt, a = p->src_amp;
    if (p->src_kind == 1) {
        double u = ((double)level - p->src_t0) / p->src_width;
        return a * exp(-u * u);
    }
    if (p->src_kind == 2) {
        double tau = 2.0 * sqrt(log(1000.0)) / (M_PI * p->src_bw);
        double t0 = p->src_t0 > 0 ? p->src_t0 : 3.0 * tau;
        double u = (t - t0) / tau;
        return a * exp(-u * u) * sin(2.0 * M_PI * p->src_fc * (t - t0));
    }
    if (p->src_kind == 3) {
        double sg = p->src_width;
        double t0 = p->src_t0 > 0 ? p->src_t0 : 3.0 * sg;
        double u = (t - t0) / sg;
        return a * (-2.0 * u) * exp(-u * u);
    }
    if (p->src_kind == 4)   /* a given pulse: sample m is added at level m + 1 */
        return (level >= 1 && level <= p->src_nsamp) ? a * p->src_samples[level - 1] : 0.0;
    return 0.0;
}

/* exported so the source spectrum can be checked on its own */
void or_waveform(const or_problem *p, int64_t first_level, int64_t count, double *out)
{
    double dt = or_dt(p);
    int64_t n;
    for (n = 0; n < count; ++n) out[n] = waveform(p, dt, first_level + n);
}

/* Length of the dual edge centred on integer node q (half-open width 1)
 * that lies inside [0, n], in cells. */
static double clip_node(int q, int n)
{
    double lo = q - 0.5, hi = q + 0.5;
    if (lo < 0) lo = 0;
    if (hi > n) hi = n;
    return hi > lo ? hi - lo : 0.0;
}

/* Closed line integral of H in the plane x = (m + 1/2) dx around the strip
 * cells y in [y0,y1), z in [z0,z1): the rectangle through the H nodes half a
 * cell outside the metal, oriented counter-clockwise seen from +x (so the
 * integral is the +x current by Ampere's law).  Segments outside the grid
 * contribute nothing; the end nodes of a segment on a grid face count with
 * the part of their dual edge inside the grid. */
static double loop_current(const or_problem *p, const or_state *s, int m,
                           int y0, int y1, int z0, int z1)
{
    double I = 0;
    int j, k;
    /* bottom, z = z0 - 1/2, along +y: Hy(m+1/2, j, z0-1/2) */
    if (z0 - 1 >= 0)
        for (j = y0; j <= y1; ++j)
            I += s->h[1][idx(p, m, j, z0 - 1)] * clip_node(j, p->ny) * p->dy;
    /* right, y = y1 + 1/2, along +z: Hz(m+1/2, y1+1/2, k) */
    if (y1 < p->ny)
        for (k = z0; k <= z1; ++k)
            I += s->h[2][idx(p, m, y1, k)] * clip_node(k, p->nz) * p->dz;
    /* top, z = z1 + 1/2, along -y */
    if (z1 < p->nz)
        for (j = y0; j <= y1; ++j)
            I -= s->h[1][idx(p, m, j, z1)] * clip_node(j, p->ny) * p->dy;
    /* left, y = y0 - 1/2, along -z */
    if (y0 - 1 >= 0)
        for (k = z0; k <= z1; ++k)
            I -= s->h[2][idx(p, m, y0 - 1, k)] * clip_node(k, p->nz) * p->dz;
    return I;
}

/* Port voltage: minus the surface integral of Ez over the nodes of plane i
 * between the ground (z = 0) and the strip bottom (z = z0), trapezoidal in y
 * across the strip, divided by the strip width. */
static double port_voltage(const or_problem *p, const or_state *s, int i, int y0, int y1, int z0)
{
    double acc = 0;
    int j, k;
    for (j = y0; j <= y1; ++j) {
        double wj = (j == y0 || j == y1) ? 0.5 : 1.0;
        double col = 0;
        for (k = 0; k < z0; ++k) col += s->e[2][idx(p, i, j, k)] * p->dz;
        acc += wj * col * p->dy;
    }
    return -acc / ((y1 - y0) * p->dy);
}

static void sample_probes(const or_problem *p, or_state *s, double dt, int64_t n)
{
    int q, f, sig;
    int nprobe = p->nport + p->npoint;
    for (q = 0; q < nprobe; ++q) {
        double val[2];
        if (q < p->nport) {
            const int32_t *d = p->ports + 6 * q;
            int ip = d[0], dir = d[1], y0 = d[2], y1 = d[3], z0 = d[4], z1 = d[5];
            val[0] = port_voltage(p, s, ip, y0, y1, z0);
            val[1] = dir * 0.5 * (loop_current(p, s, ip - 1, y0, y1, z0, z1) +
                                  loop_current(p, s, ip, y0, y1, z0, z1));
        } else {
            const int32_t *d = p->points + 4 * (q - p->nport);
            int comp = d[0];
            size_t id = idx(p, d[1], d[2], d[3]);
            val[0] = comp < 3 ? s->e[comp][id] : s->h[comp - 3][id];
            val[1] = 0.0;
        }
        for (sig = 0; sig < 2; ++sig) {
            /* V (and point values) at t = n dt, I at t = (n - 1/2) dt */
            double tn = sig == 0 ? (double)n : (double)n - 0.5;
            if (s->hist && n - 1 < s->hist_len)
                s->hist[((size_t)q * 2 + sig) * s->hist_len + (n - 1)] = val[sig];
            for (f = 0; f < p->nf; ++f) {
                double cyc = p->freqs[f] * dt * tn;
                double ph = 2.0 * M_PI * (cyc - floor(cyc));
                double *a = s->acc + (((size_t)q * 2 + sig) * p->nf + f) * 2;
                a[0] += val[sig] * cos(ph) * dt;
                a[1] -= val[sig] * sin(ph) * dt;
            }
        }
    }
}

#define PSI(name) s->psi[name]
enum { P_HXY, P_HXZ, P_HYZ, P_HYX, P_HZX, P_HZY, P_EXY, P_EXZ, P_EYZ, P_EYX, P_EZX, P_EZY };

static void update_h(const or_problem *p, or_state *s, double dt, double *wh)
{
    const double ch = dt / mu0_of(p);
    const double dx = p->dx, dy = p->dy, dz = p->dz;
    double *Ex = s->e[0], *Ey = s->e[1], *Ez = s->e[2];
    double *Hx = s->h[0], *Hy = s->h[1], *Hz = s->h[2];
    int i, j, k;
    double w = 0;
    /* Hx(i, j+1/2, k+1/2) */
#pragma omp parallel for private(i, j) reduction(+ : w) schedule(static)
    for (k = 0; k < p->nz; ++k)
        for (j = 0; j < p->ny; ++j)
            for (i = 0; i <= p->nx; ++i) {
                size_t id = idx(p, i, j, k);
                double dEz_dy = (Ez[idx(p, i, j + 1, k)] - Ez[id]) / dy;
                double dEy_dz = (Ey[idx(p, i, j, k + 1)] - Ey[id]) / dz;
                double py = 0, pz = 0;
                if (s->inH[1][j]) py = PSI(P_HXY)[id] = s->bH[1][j] * PSI(P_HXY)[id] + s->cH[1][j] * dEz_dy;
                if (s->inH[2][k]) pz = PSI(P_HXZ)[id] = s->bH[2][k] * PSI(P_HXZ)[id] + s->cH[2][k] * dEy_dz;
                double old = Hx[id];
                Hx[id] = old - ch * (dEz_dy * s->ikH[1][j] - dEy_dz * s->ikH[2][k] + py - pz);
                w += old * Hx[id];
            }
    /* Hy(i+1/2, j, k+1/2) */
#pragma omp parallel for private(i, j) reduction(+ : w) schedule(static)
    for (k = 0; k < p->nz; ++k)
        for (j = 0; j <= p->ny; ++j)
            for (i = 0; i < p->nx; ++i) {
                size_t id = idx(p, i, j, k);
                double dEx_dz = (Ex[idx(p, i, j, k + 1)] - Ex[id]) / dz;
                double dEz_dx = (Ez[idx(p, i + 1, j, k)] - Ez[id]) / dx;
                double pz = 0, px = 0;
                if (s->inH[2][k]) pz = PSI(P_HYZ)[id] = s->bH[2][k] * PSI(P_HYZ)[id] + s->cH[2][k] * dEx_dz;
                if (s->inH[0][i]) px = PSI(P_HYX)[id] = s->bH[0][i] * PSI(P_HYX)[id] + s->cH[0][i] * dEz_dx;
                double old = Hy[id];
                Hy[id] = old - ch * (dEx_dz * s->ikH[2][k] - dEz_dx * s->ikH[0][i] + pz - px);
                w += old * Hy[id];
            }
    /* Hz(i+1/2, j+1/2, k) */
#pragma omp parallel for private(i, j) reduction(+ : w) schedule(static)
    for (k = 0; k <= p->nz; ++k)
        for (j = 0; j < p->ny; ++j)
            for (i = 0; i < p->nx; ++i) {
                size_t id = idx(p, i, j, k);
                double dEy_dx = (Ey[idx(p, i + 1, j, k)] - Ey[id]) / dx;
                double dEx_dy = (Ex[idx(p, i, j + 1, k)] - Ex[id]) / dy;
                double px = 0, py = 0;
                if (s->inH[0][i]) px = PSI(P_HZX)[id] = s->bH[0][i] * PSI(P_HZX)[id] + s->cH[0][i] * dEy_dx;
                if (s->inH[1][j]) py = PSI(P_HZY)[id] = s->bH[1][j] * PSI(P_HZY)[id] + s->cH[1][j] * dEx_dy;
                double old = Hz[id];
                Hz[id] = old - ch * (dEy_dx * s->ikH[0][i] - dEx_dy * s->ikH[1][j] + px - py);
                w += old * Hz[id];
            }
    *wh = w;
}

static void update_e(const or_problem *p, or_state *s)
{
    const double dx = p->dx, dy = p->dy, dz = p->dz;
    double *Ex = s->e[0], *Ey = s->e[1], *Ez = s->e[2];
    int i, j, k;
    /* Ex(i+1/2, j, k) */
#pragma omp parallel for private(i, j) schedule(static)
    for (k = 0; k <= p->nz; ++k)
        for (j = 0; j <= p->ny; ++j)
            for (i = 0; i < p->nx; ++i) {
                size_t id = idx(p, i, j, k);
                double dHz_dy = (hval(p, s, 2, i, j, k) - hval(p, s, 2, i, j - 1, k)) / dy;
                double dHy_dz = (hval(p, s, 1, i, j, k) - hval(p, s, 1, i, j, k - 1)) / dz;
                double py = 0, pz = 0;
                if (s->inE[1][j]) py = PSI(P_EXY)[id] = s->bE[1][j] * PSI(P_EXY)[id] + s->cE[1][j] * dHz_dy;
                if (s->inE[2][k]) pz = PSI(P_EXZ)[id] = s->bE[2][k] * PSI(P_EXZ)[id] + s->cE[2][k] * dHy_dz;
                Ex[id] = s->ca[0][id] * Ex[id] +
                         s->cb[0][id] * (dHz_dy * s->ikE[1][j] - dHy_dz * s->ikE[2][k] + py - pz);
            }
    /* Ey(i, j+1/2, k) */
#pragma omp parallel for private(i, j) schedule(static)
    for (k = 0; k <= p->nz; ++k)
        for (j = 0; j < p->ny; ++j)
            for (i = 0; i <= p->nx; ++i) {
                size_t id = idx(p, i, j, k);
                double dHx_dz = (hval(p, s, 0, i, j, k) - hval(p, s, 0, i, j, k - 1)) / dz;
                double dHz_dx = (hval(p, s, 2, i, j, k) - hval(p, s, 2, i - 1, j, k)) / dx;
                double pz = 0, px = 0;
                if (s->inE[2][k]) pz = PSI(P_EYZ)[id] = s->bE[2][k] * PSI(P_EYZ)[id] + s->cE[2][k] * dHx_dz;
                if (s->inE[0][i]) px = PSI(P_EYX)[id] = s->bE[0][i] * PSI(P_EYX)[id] + s->cE[0][i] * dHz_dx;
                Ey[id] = s->ca[1][id] * Ey[id] +
                         s->cb[1][id] * (dHx_dz * s->ikE[2][k] - dHz_dx * s->ikE[0][i] + pz - px);
            }
    /* Ez(i, j, k+1/2) */
#pragma omp parallel for private(i, j) schedule(static)
    for (k = 0; k < p->nz; ++k)
        for (j = 0; j <= p->ny; ++j)
            for (i = 0; i <= p->nx; ++i) {
                size_t id = idx(p, i, j, k);
                double dHy_dx = (hval(p, s, 1, i, j, k) - hval(p, s, 1, i - 1, j, k)) / dx;
                double dHx_dy = (hval(p, s, 0, i, j, k) - hval(p, s, 0, i, j - 1, k)) / dy;
                double px = 0, py = 0;
                if (s->inE[0][i]) px = PSI(P_EZX)[id] = s->bE[0][i] * PSI(P_EZX)[id] + s->cE[0][i] * dHy_dx;
                if (s->inE[1][j]) py = PSI(P_EZY)[id] = s->bE[1][j] * PSI(P_EZY)[id] + s->cE[1][j] * dHx_dy;
                Ez[id] = s->ca[2][id] * Ez[id] +
                         s->cb[2][id] * (dHy_dx * s->ikE[0][i] - dHx_dy * s->ikE[1][j] + px - py);
            }
}

/* Electric part of the discrete energy, sum over edges of eps E^2 / 2 times
 * the cell volume (eps recovered from Cb = dt/eps on lossless edges). */
static double energy_e(const or_problem *p, const or_state *s, double dt)
{
    double w = 0;
    int comp, i, j, k;
    for (comp = 0; comp < 3; ++comp) {
        const double *E = s->e[comp], *cb = s->cb[comp];
#pragma omp parallel for private(i, j) reduction(+ : w) schedule(static)
        for (k = 0; k <= p->nz; ++k)
            for (j = 0; j <= p->ny; ++j)
                for (i = 0; i <= p->nx; ++i) {
                    size_t id = idx(p, i, j, k);
                    if (cb[id] != 0.0) w += 0.5 * (dt / cb[id]) * E[id] * E[id];
                }
    }
    return w;
}

/* Advance nsteps steps.  Returns 0. */
int or_run(const or_problem *p, or_state *s, int64_t nsteps)
{
    double dt = or_dt(p);
    double dV = p->dx * p->dy * p->dz;
    int64_t t;
    int i, j, k;
    for (t = 0; t < nsteps; ++t) {
        int64_t n = s->step;  /* fields hold E^n, H^{n-1/2} */
        double we = s->energy ? energy_e(p, s, dt) : 0.0;
        double wh = 0;
        update_h(p, s, dt, &wh);
        if (s->energy && n < s->hist_len)
            s->energy[n] = (we + 0.5 * mu0_of(p) * wh) * dV;
        update_e(p, s);
        if (p->src_kind) {
            double v = waveform(p, dt, n + 1);
            const int32_t *b = p->src_box;
            for (k = b[4]; k <= b[5]; ++k)
                for (j = b[2]; j <= b[3]; ++j)
                    for (i = b[0]; i <= b[1]; ++i) s->e[p->src_comp][idx(p, i, j, k)] += v;
        }
        s->step = n + 1;
        sample_probes(p, s, dt, n + 1);
    }
    return 0;
}

/* Size of the OpenMP team the loops above run on, and a way to change it
 * (timing of the oracle at a stated thread count; no effect on results,
 * since every parallel loop writes disjoint cells and the reductions only
 * feed the optional energy record). */
int or_max_threads(void) { return omp_get_max_threads(); }
void or_set_threads(int n)
{
    if (n > 0) omp_set_num_threads(n);
}
