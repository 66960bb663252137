/*
 * Plain FP64 CPU oracle for the single-level BoxLib hot path.
 *
 * TEST INFRASTRUCTURE ONLY: this file is compiled into liboracle.so and is
 * called by the tests, by the package smoke check and by the CPU-baseline leg
 * of the benchmark.  The product library never links, loads or calls it.
 *
 * Every routine is written as the plain definition of what it computes, with
 * no tiling, blocking, vectorisation or reordering, in the operand order that
 * the comments state.  Build with -O2 -ffp-contract=off (no FMA contraction)
 * so the rounding of every cell update is exactly the one written here.
 *
 * Data model (the oracle's own, independent of the product library):
 *   - a Box is six ints {lo[3], hi[3]}, inclusive cell indices (paper, Sec. 3.1:
 *     a three-dimensional Box is represented by six integers);
 *   - a FAB (FArrayBox) holds ncomp components on its box grown by ng ghost
 *     cells, stored as one contiguous array, x fastest, then y, z, then the
 *     component (paper, Sec. 3.1: multi-component data in one contiguous 1-D
 *     array reshaped as a Fortran array);
 *   - a MultiFab is nbox FABs of one level; here all FABs live in one double
 *     array and fab_off[b] is the element offset of FAB b.
 *
 * Routines:
 *   orc_fill_boundary  FillBoundary with periodic wrap (Sec. 3.1, Sec. 3.3,
 *                      Sec. 4.1): every ghost cell takes the valid value at its
 *                      periodically wrapped index if some box covers it.
 *   orc_heat_step      forward-Euler step of the heat equation with
 *                      second-order centred differences (Sec. 4.1), written as
 *                      the 7-point update.
 *   orc_heat_flux_step the same step in the paper's own form (Sec. 4.1): three
 *                      face-flux loops, then a divergence loop.
 *   orc_heat_varcoef_step  the flux form with a variable diffusion coefficient:
 *                      each face's coefficient is the mean of its two cells.
 *   orc_heat8_step     forward-Euler heat step with the 8th-order centred second
 *                      difference (9 cells per axis, 4 ghost layers).
 *   orc_gsrb_color     one colour of a red-black Gauss-Seidel sweep for the
 *                      7-point discrete Poisson problem -L_h phi = f.
 *   orc_residual       r = f + L_h phi per valid cell (FP64).
 *   orc_restrict_residual  multigrid restriction: each cell of the coarsened
 *                      level takes the mean of the residuals of its 8 cells.
 *   orc_prolong_add    multigrid prolongation: each fine cell adds the value of
 *                      the coarse cell that contains it.
 *   orc_heat_window    n heat steps on a cube window of a fully periodic global
 *                      array, returning the centre value (used to check single
 *                      outputs of very large runs one by one).
 *   orc_fsum           exactly rounded sum of an array (the reductions' and the
 *                      residual norm's sum).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads the box loops may use (OpenMP over boxes only: each box is updated
 * by one thread in the plain order, so results do not depend on the count). */
int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Thread count of the box loops from here on (n > 0); used to time the oracle
 * on one thread beside its all-cores run. */
void orc_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

typedef struct {
  int nx, ny, nz;      /* grown extents */
  int glo[3];          /* grown lower corner (global index) */
} fab_geom;

static fab_geom geom_of(const int* box, int ng) {
  fab_geom g;
  g.glo[0] = box[0] - ng;
  g.glo[1] = box[1] - ng;
  g.glo[2] = box[2] - ng;
  g.nx = box[3] - box[0] + 1 + 2 * ng;
  g.ny = box[4] - box[1] + 1 + 2 * ng;
  g.nz = box[5] - box[2] + 1 + 2 * ng;
  return g;
}

/* element index of global cell (i,j,k), component comp, inside a FAB */
static int64_t fab_index(const fab_geom* g, int comp, int i, int j, int k) {
  int64_t li = i - g->glo[0], lj = j - g->glo[1], lk = k - g->glo[2];
  return (((int64_t)comp * g->nz + lk) * g->ny + lj) * g->nx + li;
}

static int floor_mod(int a, int n) {
  int r = a % n;
  return r < 0 ? r + n : r;
}

static int floor_half(int a) { return (a - floor_mod(a, 2)) / 2; }

/*
 * Owner map of the level: owner[(k*N1 + j)*N0 + i] = index of the box whose
 * valid region holds domain cell (i,j,k), or -1.  Returns -1 if two boxes
 * overlap or a box leaves the domain (the grids of a level are
 * non-intersecting, Sec. 3).
 */
int orc_owner_map(int nbox, const int* boxes, const int* domain, int32_t* owner) {
  int N0 = domain[3] - domain[0] + 1, N1 = domain[4] - domain[1] + 1, N2 = domain[5] - domain[2] + 1;
  int64_t ncell = (int64_t)N0 * N1 * N2;
  for (int64_t q = 0; q < ncell; ++q) owner[q] = -1;
  for (int b = 0; b < nbox; ++b) {
    const int* bx = boxes + 6 * b;
    for (int d = 0; d < 3; ++d)
      if (bx[d] < domain[d] || bx[3 + d] > domain[3 + d] || bx[d] > bx[3 + d]) return -1;
    for (int k = bx[2]; k <= bx[5]; ++k)
      for (int j = bx[1]; j <= bx[4]; ++j)
        for (int i = bx[0]; i <= bx[3]; ++i) {
          int64_t q = ((int64_t)(k - domain[2]) * N1 + (j - domain[1])) * N0 + (i - domain[0]);
          if (owner[q] >= 0) return -1;
          owner[q] = b;
        }
  }
  return 0;
}

/*
 * FillBoundary(mf, scomp, ncomp).  Plain definition: assemble the global array
 * G of one component from all valid regions; then every ghost cell p of every
 * FAB takes G(p') where p' is p wrapped modulo the domain extent along each
 * periodic axis, provided p' lies inside the domain and inside some box.  Ghost
 * cells that no box covers (outside a non-periodic domain, or in a hole of a
 * non-covering box list) are left untouched.
 *   G      : scratch, one domain-sized double array
 *   owner  : the owner map from orc_owner_map
 */
void orc_fill_boundary(int nbox, const int* boxes, const int* domain, const int* periodic,
                       int ng, int scomp, int ncomp, double* data, const int64_t* fab_off,
                       double* G, const int32_t* owner) {
  int N[3], lo[3];
  for (int d = 0; d < 3; ++d) {
    lo[d] = domain[d];
    N[d] = domain[3 + d] - domain[d] + 1;
  }
  for (int comp = scomp; comp < scomp + ncomp; ++comp) {
    /* gather the valid regions into G */
#pragma omp parallel for schedule(dynamic)
    for (int b = 0; b < nbox; ++b) {
      const int* bx = boxes + 6 * b;
      fab_geom g = geom_of(bx, ng);
      const double* fab = data + fab_off[b];
      for (int k = bx[2]; k <= bx[5]; ++k)
        for (int j = bx[1]; j <= bx[4]; ++j)
          for (int i = bx[0]; i <= bx[3]; ++i) {
            int64_t q = ((int64_t)(k - lo[2]) * N[1] + (j - lo[1])) * N[0] + (i - lo[0]);
            G[q] = fab[fab_index(&g, comp, i, j, k)];
          }
    }
    /* every ghost cell of every FAB */
#pragma omp parallel for schedule(dynamic)
    for (int b = 0; b < nbox; ++b) {
      const int* bx = boxes + 6 * b;
      fab_geom g = geom_of(bx, ng);
      double* fab = data + fab_off[b];
      for (int k = bx[2] - ng; k <= bx[5] + ng; ++k)
        for (int j = bx[1] - ng; j <= bx[4] + ng; ++j)
          for (int i = bx[0] - ng; i <= bx[3] + ng; ++i) {
            int inside = i >= bx[0] && i <= bx[3] && j >= bx[1] && j <= bx[4] && k >= bx[2] && k <= bx[5];
            if (inside) continue;
            int p[3] = {i, j, k};
            int ok = 1;
            for (int d = 0; d < 3; ++d) {
              if (periodic[d]) p[d] = lo[d] + floor_mod(p[d] - lo[d], N[d]);
              if (p[d] < lo[d] || p[d] >= lo[d] + N[d]) ok = 0;
            }
            if (!ok) continue;
            int64_t q = ((int64_t)(p[2] - lo[2]) * N[1] + (p[1] - lo[1])) * N[0] + (p[0] - lo[0]);
            if (owner[q] < 0) continue;
            fab[fab_index(&g, comp, i, j, k)] = G[q];
          }
    }
  }
}

/*
 * One forward-Euler heat step on the valid cells of every FAB (Sec. 4.1),
 * reading u_old (whose ghosts must have been filled) and writing u_new:
 *   s     = ((u[i-1] + u[i+1]) + (u[j-1] + u[j+1])) + (u[k-1] + u[k+1])
 *   u_new = u + c * (s - 6 u),   c = dt / dx^2
 * Ghost cells of u_new are not written.
 */
void orc_heat_step(int nbox, const int* boxes, int ng, int ncomp, const double* uold,
                   double* unew, const int64_t* fab_off, double c) {
#pragma omp parallel for schedule(dynamic)
  for (int b = 0; b < nbox; ++b) {
    const int* bx = boxes + 6 * b;
    fab_geom g = geom_of(bx, ng);
    const double* u = uold + fab_off[b];
    double* v = unew + fab_off[b];
    for (int comp = 0; comp < ncomp; ++comp)
      for (int k = bx[2]; k <= bx[5]; ++k)
        for (int j = bx[1]; j <= bx[4]; ++j)
          for (int i = bx[0]; i <= bx[3]; ++i) {
            double uc = u[fab_index(&g, comp, i, j, k)];
            double sx = u[fab_index(&g, comp, i - 1, j, k)] + u[fab_index(&g, comp, i + 1, j, k)];
            double sy = u[fab_index(&g, comp, i, j - 1, k)] + u[fab_index(&g, comp, i, j + 1, k)];
            double sz = u[fab_index(&g, comp, i, j, k - 1)] + u[fab_index(&g, comp, i, j, k + 1)];
            double s = (sx + sy) + sz;
            v[fab_index(&g, comp, i, j, k)] = uc + c * (s - 6.0 * uc);
          }
  }
}

/*
 * The same heat step in the paper's own structure (Sec. 4.1): the flux of each
 * direction is computed on the faces of the box in its own loop,
 *   F^x(i-1/2) = (u[i] - u[i-1]) * inv_dx   (likewise for y and z),
 * and a fourth loop forms the divergence and updates
 *   u_new = u + dt * ( (F^x(i+1/2) - F^x(i-1/2)) * inv_dx + (y) + (z) ).
 * inv_dx = 1/dx is formed once by the caller, as c = dt/dx^2 is for the
 * 7-point form.  Algebraically identical to orc_heat_step; rounding differs.
 * Returns -1 if the flux scratch cannot be allocated.
 */
int orc_heat_flux_step(int nbox, const int* boxes, int ng, int ncomp, const double* uold,
                       double* unew, const int64_t* fab_off, double dt, double inv_dx) {
  for (int b = 0; b < nbox; ++b) {
    const int* bx = boxes + 6 * b;
    fab_geom g = geom_of(bx, ng);
    int ex = bx[3] - bx[0] + 1, ey = bx[4] - bx[1] + 1, ez = bx[5] - bx[2] + 1;
    /* face-centred flux arrays: nodal in their own direction */
    double* fx = (double*)malloc(sizeof(double) * (size_t)(ex + 1) * ey * ez);
    double* fy = (double*)malloc(sizeof(double) * (size_t)ex * (ey + 1) * ez);
    double* fz = (double*)malloc(sizeof(double) * (size_t)ex * ey * (ez + 1));
    if (!fx || !fy || !fz) {
      free(fx); free(fy); free(fz);
      return -1;
    }
    const double* u = uold + fab_off[b];
    double* v = unew + fab_off[b];
    for (int comp = 0; comp < ncomp; ++comp) {
      for (int k = 0; k < ez; ++k)
        for (int j = 0; j < ey; ++j)
          for (int i = 0; i <= ex; ++i) {
            int gi = bx[0] + i, gj = bx[1] + j, gk = bx[2] + k;
            fx[((size_t)k * ey + j) * (ex + 1) + i] =
                (u[fab_index(&g, comp, gi, gj, gk)] - u[fab_index(&g, comp, gi - 1, gj, gk)]) * inv_dx;
          }
      for (int k = 0; k < ez; ++k)
        for (int j = 0; j <= ey; ++j)
          for (int i = 0; i < ex; ++i) {
            int gi = bx[0] + i, gj = bx[1] + j, gk = bx[2] + k;
            fy[((size_t)k * (ey + 1) + j) * ex + i] =
                (u[fab_index(&g, comp, gi, gj, gk)] - u[fab_index(&g, comp, gi, gj - 1, gk)]) * inv_dx;
          }
      for (int k = 0; k <= ez; ++k)
        for (int j = 0; j < ey; ++j)
          for (int i = 0; i < ex; ++i) {
            int gi = bx[0] + i, gj = bx[1] + j, gk = bx[2] + k;
            fz[((size_t)k * ey + j) * ex + i] =
                (u[fab_index(&g, comp, gi, gj, gk)] - u[fab_index(&g, comp, gi, gj, gk - 1)]) * inv_dx;
          }
      for (int k = 0; k < ez; ++k)
        for (int j = 0; j < ey; ++j)
          for (int i = 0; i < ex; ++i) {
            int gi = bx[0] + i, gj = bx[1] + j, gk = bx[2] + k;
            double dfx = (fx[((size_t)k * ey + j) * (ex + 1) + i + 1] - fx[((size_t)k * ey + j) * (ex + 1) + i]) * inv_dx;
            double dfy = (fy[((size_t)k * (ey + 1) + j + 1) * ex + i] - fy[((size_t)k * (ey + 1) + j) * ex + i]) * inv_dx;
            double dfz = (fz[((size_t)(k + 1) * ey + j) * ex + i] - fz[((size_t)k * ey + j) * ex + i]) * inv_dx;
            int64_t q = fab_index(&g, comp, gi, gj, gk);
            v[q] = u[q] + dt * ((dfx + dfy) + dfz);
          }
    }
    free(fx);
    free(fy);
    free(fz);
  }
  return 0;
}

/*
 * Heat step with a variable diffusion coefficient beta, a cell-centred field
 * with the layout of u whose ghost cells are filled, in the flux form of
 * Sec. 4.1 extended to du/dt = div(beta grad u): on each face the coefficient
 * is the mean of the two cells it separates,
 *   b(i-1/2) = 0.5 * (beta[i-1] + beta[i]),
 *   F^x(i-1/2) = b(i-1/2) * ((u[i] - u[i-1]) * inv_dx)     (likewise y, z),
 * then, per cell,
 *   u_new = u + dt * ((dFx + dFy) + dFz),   dFx = (F^x(i+1/2) - F^x(i-1/2)) * inv_dx,
 * with inv_dx = 1/dx formed once by the caller.
 * With beta = 1 every b is exactly 1 and the result is orc_heat_flux_step's.
 * Written per cell: each face flux is the same expression from either side.
 */
static double vflux(const double* u, const double* bt, int64_t lo, int64_t hi, double inv_dx) {
  const double b = 0.5 * (bt[lo] + bt[hi]);
  return b * ((u[hi] - u[lo]) * inv_dx);
}

void orc_heat_varcoef_step(int nbox, const int* boxes, int ng, int ncomp, const double* uold,
                           const double* beta, double* unew, const int64_t* fab_off, double dt, double inv_dx) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int b = 0; b < nbox; ++b) {
    const int* bx = boxes + 6 * b;
    fab_geom g = geom_of(bx, ng);
    const double* u = uold + fab_off[b];
    const double* bt = beta + fab_off[b];
    double* v = unew + fab_off[b];
    for (int comp = 0; comp < ncomp; ++comp)
      for (int k = bx[2]; k <= bx[5]; ++k)
        for (int j = bx[1]; j <= bx[4]; ++j)
          for (int i = bx[0]; i <= bx[3]; ++i) {
            const int64_t c = fab_index(&g, comp, i, j, k);
            const double fxm = vflux(u, bt, fab_index(&g, comp, i - 1, j, k), c, inv_dx);
            const double fxp = vflux(u, bt, c, fab_index(&g, comp, i + 1, j, k), inv_dx);
            const double fym = vflux(u, bt, fab_index(&g, comp, i, j - 1, k), c, inv_dx);
            const double fyp = vflux(u, bt, c, fab_index(&g, comp, i, j + 1, k), inv_dx);
            const double fzm = vflux(u, bt, fab_index(&g, comp, i, j, k - 1), c, inv_dx);
            const double fzp = vflux(u, bt, c, fab_index(&g, comp, i, j, k + 1), inv_dx);
            const double dfx = (fxp - fxm) * inv_dx, dfy = (fyp - fym) * inv_dx, dfz = (fzp - fzm) * inv_dx;
            v[c] = u[c] + dt * ((dfx + dfy) + dfz);
          }
  }
}

/*
 * One colour of a red-black Gauss-Seidel sweep for -L_h phi = f with the
 * 7-point Laplacian L_h phi = (sum of 6 neighbours - 6 phi) / h2.  The colour
 * of cell (i,j,k) is the parity of i+j+k in global indices (0 = red, 1 =
 * black).  Each cell of the colour is solved for exactly, in place:
 *   phi = ((((phi[i-1] + phi[i+1]) + (phi[j-1] + phi[j+1])) + (phi[k-1] + phi[k+1]))
 *          + h2 * f) * inv6,      inv6 = 1/6 rounded once by the caller.
 * Cells of one colour only read cells of the other colour (or ghosts), so the
 * in-place update is independent of the visiting order.
 */
void orc_gsrb_color(int nbox, const int* boxes, int ng, double* phi, const double* f,
                    const int64_t* fab_off, double h2, double inv6, int color) {
#pragma omp parallel for schedule(dynamic)
  for (int b = 0; b < nbox; ++b) {
    const int* bx = boxes + 6 * b;
    fab_geom g = geom_of(bx, ng);
    double* p = phi + fab_off[b];
    const double* fb = f + fab_off[b];
    for (int k = bx[2]; k <= bx[5]; ++k)
      for (int j = bx[1]; j <= bx[4]; ++j)
        for (int i = bx[0]; i <= bx[3]; ++i) {
          if (floor_mod(i + j + k, 2) != color) continue;
          double sx = p[fab_index(&g, 0, i - 1, j, k)] + p[fab_index(&g, 0, i + 1, j, k)];
          double sy = p[fab_index(&g, 0, i, j - 1, k)] + p[fab_index(&g, 0, i, j + 1, k)];
          double sz = p[fab_index(&g, 0, i, j, k - 1)] + p[fab_index(&g, 0, i, j, k + 1)];
          int64_t q = fab_index(&g, 0, i, j, k);
          p[q] = (((sx + sy) + sz) + h2 * fb[q]) * inv6;
        }
  }
}

/*
 * Heat step with the 8th-order centred second difference along each axis
 * (span 9 cells: the stencil width of Sec. 4.2's application, here on the
 * heat equation).  With p_m = u[i-m] + u[i+m] along an axis,
 *   D = ((A1*p1 + A2*p2) + A3*p3) + A4*p4,
 *   u_new = u + c * (((Dx + Dy) + Dz) + A0X3*u),
 * A1 = 8/5, A2 = -1/5, A3 = 8/315, A4 = -1/560 and A0X3 = 3*(-205/72) = -205/24,
 * each rounded once; c = dt/dx^2.  Needs ng >= 4 and filled ghosts.
 */
static const double H8_A1 = 8.0 / 5.0, H8_A2 = -1.0 / 5.0, H8_A3 = 8.0 / 315.0, H8_A4 = -1.0 / 560.0;
static const double H8_A0X3 = -205.0 / 24.0;

void orc_heat8_step(int nbox, const int* boxes, int ng, int ncomp, const double* uold, double* unew,
                    const int64_t* fab_off, double c) {
#pragma omp parallel for schedule(dynamic)
  for (int b = 0; b < nbox; ++b) {
    const int* bx = boxes + 6 * b;
    fab_geom g = geom_of(bx, ng);
    const double* u = uold + fab_off[b];
    double* v = unew + fab_off[b];
    for (int comp = 0; comp < ncomp; ++comp)
      for (int k = bx[2]; k <= bx[5]; ++k)
        for (int j = bx[1]; j <= bx[4]; ++j)
          for (int i = bx[0]; i <= bx[3]; ++i) {
            double p[3][5];
            for (int m = 1; m <= 4; ++m) {
              p[0][m] = u[fab_index(&g, comp, i - m, j, k)] + u[fab_index(&g, comp, i + m, j, k)];
              p[1][m] = u[fab_index(&g, comp, i, j - m, k)] + u[fab_index(&g, comp, i, j + m, k)];
              p[2][m] = u[fab_index(&g, comp, i, j, k - m)] + u[fab_index(&g, comp, i, j, k + m)];
            }
            double D[3];
            for (int d = 0; d < 3; ++d)
              D[d] = ((H8_A1 * p[d][1] + H8_A2 * p[d][2]) + H8_A3 * p[d][3]) + H8_A4 * p[d][4];
            const int64_t q = fab_index(&g, comp, i, j, k);
            v[q] = u[q] + c * (((D[0] + D[1]) + D[2]) + H8_A0X3 * u[q]);
          }
  }
}

/*
 * Residual of -L_h phi = f on the valid cells, in FP64:
 *   r = f + (s - 6 phi) / h2,  s = ((phi[i-1]+phi[i+1]) + (phi[j-1]+phi[j+1])) + (phi[k-1]+phi[k+1])
 * written box after box, each box in (k, j, i) order, into r_out.
 */
static double residual_at(const double* p, const double* fb, const fab_geom* g, int i, int j, int k, double h2) {
  double sx = p[fab_index(g, 0, i - 1, j, k)] + p[fab_index(g, 0, i + 1, j, k)];
  double sy = p[fab_index(g, 0, i, j - 1, k)] + p[fab_index(g, 0, i, j + 1, k)];
  double sz = p[fab_index(g, 0, i, j, k - 1)] + p[fab_index(g, 0, i, j, k + 1)];
  int64_t q = fab_index(g, 0, i, j, k);
  return fb[q] + (((sx + sy) + sz) - 6.0 * p[q]) / h2;
}

void orc_residual(int nbox, const int* boxes, int ng, const double* phi, const double* f,
                  const int64_t* fab_off, double h2, double* r_out) {
  int64_t n = 0;
  for (int b = 0; b < nbox; ++b) {
    const int* bx = boxes + 6 * b;
    fab_geom g = geom_of(bx, ng);
    const double* p = phi + fab_off[b];
    const double* fb = f + fab_off[b];
    for (int k = bx[2]; k <= bx[5]; ++k)
      for (int j = bx[1]; j <= bx[4]; ++j)
        for (int i = bx[0]; i <= bx[3]; ++i) r_out[n++] = residual_at(p, fb, &g, i, j, k, h2);
  }
}

/*
 * Multigrid restriction of the residual, cell-centred, refinement ratio 2.
 * Coarse box b is fine box b coarsened: lo/2 .. (hi+1)/2 - 1, every fine lo
 * and extent even.  Coarse cell (I,J,K) covers fine cells (2I+a, 2J+b, 2K+c),
 * a, b, c in {0, 1}; it takes
 *   fc = (sum of their residuals r = f + L_h phi) * 0.125,
 * the sum taken in the order c, then b, then a (lower child first), starting
 * from the first child's residual.  phi's ghost cells must be filled.
 */
void orc_restrict_residual(int nbox, const int* fboxes, const int* cboxes, int ng, const double* phi,
                           const double* f, const int64_t* ffab_off, double* fc, const int64_t* cfab_off,
                           double h2) {
#pragma omp parallel for schedule(dynamic)
  for (int b = 0; b < nbox; ++b) {
    const int* fbx = fboxes + 6 * b;
    const int* cbx = cboxes + 6 * b;
    fab_geom gf = geom_of(fbx, ng), gc = geom_of(cbx, ng);
    const double* p = phi + ffab_off[b];
    const double* fb = f + ffab_off[b];
    double* out = fc + cfab_off[b];
    for (int K = cbx[2]; K <= cbx[5]; ++K)
      for (int J = cbx[1]; J <= cbx[4]; ++J)
        for (int I = cbx[0]; I <= cbx[3]; ++I) {
          double acc = 0.0;
          int first = 1;
          for (int c = 0; c < 2; ++c)
            for (int bb = 0; bb < 2; ++bb)
              for (int a = 0; a < 2; ++a) {
                double r = residual_at(p, fb, &gf, 2 * I + a, 2 * J + bb, 2 * K + c, h2);
                acc = first ? r : acc + r;
                first = 0;
              }
          out[fab_index(&gc, 0, I, J, K)] = acc * 0.125;
        }
  }
}

/*
 * Multigrid prolongation, piecewise constant: every valid cell (i,j,k) of fine
 * box b adds the value of cell (floor(i/2), floor(j/2), floor(k/2)) of coarse
 * box b (the fine box coarsened, as for the restriction).
 */
void orc_prolong_add(int nbox, const int* fboxes, const int* cboxes, int ng, double* phi,
                     const int64_t* ffab_off, const double* pc, const int64_t* cfab_off) {
#pragma omp parallel for schedule(dynamic)
  for (int b = 0; b < nbox; ++b) {
    const int* fbx = fboxes + 6 * b;
    const int* cbx = cboxes + 6 * b;
    fab_geom gf = geom_of(fbx, ng), gc = geom_of(cbx, ng);
    double* p = phi + ffab_off[b];
    const double* c = pc + cfab_off[b];
    for (int k = fbx[2]; k <= fbx[5]; ++k)
      for (int j = fbx[1]; j <= fbx[4]; ++j)
        for (int i = fbx[0]; i <= fbx[3]; ++i)
          p[fab_index(&gf, 0, i, j, k)] += c[fab_index(&gc, 0, floor_half(i), floor_half(j), floor_half(k))];
  }
}

/*
 * n heat steps on a cube window of edge 2n+1 (x fastest) cut from a fully
 * periodic, fully covered domain around one cell: step s updates the cells at
 * distance <= n-s-1 from the centre from those at distance <= n-s, with the
 * same per-cell expression as orc_heat_step.  After n steps only the centre
 * cell remains; its value is returned.  w is modified (used as the state) and
 * tmp must hold as many doubles as w.
 */
double orc_heat_window(double* w, double* tmp, int n, double c) {
  int e = 2 * n + 1;
  double* a = w;
  double* bb = tmp;
  for (int s = 0; s < n; ++s) {
    int lo = s + 1, hi = e - 2 - s; /* cells still computable after this step */
    for (int k = lo; k <= hi; ++k)
      for (int j = lo; j <= hi; ++j)
        for (int i = lo; i <= hi; ++i) {
          int64_t q = ((int64_t)k * e + j) * e + i;
          double uc = a[q];
          double sx = a[q - 1] + a[q + 1];
          double sy = a[q - e] + a[q + e];
          double sz = a[q - (int64_t)e * e] + a[q + (int64_t)e * e];
          double s6 = (sx + sy) + sz;
          bb[q] = uc + c * (s6 - 6.0 * uc);
        }
    double* t = a;
    a = bb;
    bb = t;
  }
  return a[((int64_t)n * e + n) * e + n];
}

/*
 * Exactly rounded sum of n finite doubles: the reductions' definition (Sec. 3.1
 * names the MultiFab sum; the oracle fixes it as the real sum of the values,
 * rounded once to the nearest double, ties to even, so that it depends on
 * neither order nor decomposition).  Method: Shewchuk's adaptive expansions
 * ("Adaptive Precision Floating-Point Arithmetic and Fast Robust Geometric
 * Predicates", 1997).  The running sum is held exactly as a list of
 * non-overlapping partials of increasing magnitude; adding a value walks the
 * list with an error-free two-sum (hi = x + y rounded, lo = the exact rounding
 * error), keeping every non-zero error as a partial.  The result is the
 * partials added from the largest down, stopping at the first inexact
 * addition, with one correction so that a tie between two doubles, decided by
 * the partials below, rounds the right way.
 *
 * Each thread sums a contiguous chunk into its own partials; the threads'
 * partials are then added, exactly, into one list.  Since every step is exact
 * the result does not depend on the thread count.  Partials are non-overlapping
 * bit ranges inside the 2098-bit range of finite doubles, so there are never
 * more than ORC_MAX_PARTIALS of them.  Returns NaN if a value or a partial is
 * not finite (inputs here are residuals and states, far from overflow).
 */
#define ORC_MAX_PARTIALS 2112

static int partials_add(double* p, int np, double x) {
  int m = 0;
  for (int j = 0; j < np; ++j) {
    double y = p[j];
    if ((x < 0 ? -x : x) < (y < 0 ? -y : y)) {
      double t = x;
      x = y;
      y = t;
    }
    double hi = x + y;
    double lo = y - (hi - x); /* exact: |x| >= |y| */
    if (lo != 0.0) p[m++] = lo;
    x = hi;
  }
  p[m++] = x;
  return m;
}

static double partials_round(const double* p, int np) {
  if (np == 0) return 0.0;
  int n = np;
  double hi = p[--n], lo = 0.0;
  while (n > 0) {
    double x = hi, y = p[--n];
    hi = x + y;
    lo = y - (hi - x);
    if (lo != 0.0) break;
  }
  /* hi + lo is exact and lo is half an ulp of hi or less; if the partials still
   * below point the same way as lo, a tie in hi + lo must round away from hi */
  if (n > 0 && ((lo < 0 && p[n - 1] < 0) || (lo > 0 && p[n - 1] > 0))) {
    double y = lo * 2.0, x = hi + y;
    if (y == x - hi) hi = x;
  }
  return hi;
}

double orc_fsum(const double* v, int64_t n) {
  int nt = orc_num_threads();
  if (nt < 1) nt = 1;
  if ((int64_t)nt > n / 65536 + 1) nt = (int)(n / 65536 + 1);
  double* all = (double*)malloc(sizeof(double) * (size_t)nt * ORC_MAX_PARTIALS);
  int* cnt = (int*)calloc((size_t)nt, sizeof(int));
  int bad = 0;
  if (!all || !cnt) {
    free(all);
    free(cnt);
    return 0.0 / 0.0;
  }
#pragma omp parallel for schedule(static, 1) num_threads(nt) reduction(| : bad)
  for (int t = 0; t < nt; ++t) {
    int64_t a = n * t / nt, b = n * (t + 1) / nt;
    double* p = all + (size_t)t * ORC_MAX_PARTIALS;
    int np = 0;
    for (int64_t i = a; i < b; ++i) {
      double x = v[i];
      if (x - x != 0.0) { /* inf or NaN */
        bad = 1;
        break;
      }
      np = partials_add(p, np, x);
      if (p[np - 1] - p[np - 1] != 0.0) {
        bad = 1;
        break;
      }
    }
    cnt[t] = np;
  }
  double res = 0.0 / 0.0;
  if (!bad) {
    double* q = (double*)malloc(sizeof(double) * ORC_MAX_PARTIALS);
    if (q) {
      int nq = 0;
      for (int t = 0; t < nt; ++t)
        for (int j = 0; j < cnt[t]; ++j) nq = partials_add(q, nq, all[(size_t)t * ORC_MAX_PARTIALS + j]);
      res = partials_round(q, nq);
      free(q);
    }
  }
  free(all);
  free(cnt);
  return res;
}
