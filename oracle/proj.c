/*
 * Oracle parallel-beam projector P_theta and its exact transpose, FP64.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the Python oracle through ctypes; no
 * product code links it.  Shares nothing with the HIP library.
 *
 * Definition followed: Sec. 2.2, eq. ptheta2 with eq. qtheta --
 *   rho_theta(x', z) = int rho((x, y) Q_theta^T, z) dy,
 *   (x, y) Q_theta^T = (x cos t + y sin t, -x sin t + y cos t),
 * discretised as the Riemann sum the paper describes (eq. ptheta1): unit-step
 * samples y_q along the ray through detector position u_p, the volume read
 * by bilinear interpolation inside each z-slice, neighbours outside the grid
 * counting as zero.
 *
 * Layouts: vol[k][j][i] (i fastest), proj[m][k][p].
 * oracle_backproject is the transpose written as the same loops with the
 * gather turned into a scatter, so it is the exact adjoint of
 * oracle_project up to floating-point summation order.
 */
#include <math.h>
#include <stddef.h>

static double voxel(const double *slice, int nx, int ny, long i, long j)
{
    if (i < 0 || j < 0 || i >= nx || j >= ny) return 0.0;
    return slice[j * (long)nx + i];
}

static void add_voxel(double *slice, int nx, int ny, long i, long j, double v)
{
    if (i < 0 || j < 0 || i >= nx || j >= ny) return;
    slice[j * (long)nx + i] += v;
}

void oracle_project(const double *vol, int nx, int ny, int nz,
                    int nm, const double *cos_t, const double *sin_t,
                    const double *u, int nu, const double *yq, int nr,
                    double *proj)
{
    const double cx = 0.5 * (nx - 1), cy = 0.5 * (ny - 1);
    long total = (long)nm * nz;
#pragma omp parallel for schedule(static)
    for (long mk = 0; mk < total; ++mk) {
        int m = (int)(mk / nz), k = (int)(mk % nz);
        const double *slice = vol + (long)k * nx * ny;
        double c = cos_t[m], s = sin_t[m];
        for (int p = 0; p < nu; ++p) {
            double acc = 0.0;
            for (int q = 0; q < nr; ++q) {
                double X = u[p] * c + yq[q] * s;
                double Y = -u[p] * s + yq[q] * c;
                double fx = X + cx, fy = Y + cy;
                double i0 = floor(fx), j0 = floor(fy);
                double ax = fx - i0, ay = fy - j0;
                long i = (long)i0, j = (long)j0;
                acc += (1.0 - ax) * (1.0 - ay) * voxel(slice, nx, ny, i, j)
                     + ax * (1.0 - ay) * voxel(slice, nx, ny, i + 1, j)
                     + (1.0 - ax) * ay * voxel(slice, nx, ny, i, j + 1)
                     + ax * ay * voxel(slice, nx, ny, i + 1, j + 1);
            }
            proj[((long)m * nz + k) * nu + p] = acc; /* ray step dy = 1 */
        }
    }
}

void oracle_backproject(const double *proj, int nx, int ny, int nz,
                        int nm, const double *cos_t, const double *sin_t,
                        const double *u, int nu, const double *yq, int nr,
                        double *vol)
{
    const double cx = 0.5 * (nx - 1), cy = 0.5 * (ny - 1);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k) {
        double *slice = vol + (long)k * nx * ny;
        for (long t = 0; t < (long)nx * ny; ++t) slice[t] = 0.0;
        for (int m = 0; m < nm; ++m) {
            double c = cos_t[m], s = sin_t[m];
            for (int p = 0; p < nu; ++p) {
                double g = proj[((long)m * nz + k) * nu + p];
                for (int q = 0; q < nr; ++q) {
                    double X = u[p] * c + yq[q] * s;
                    double Y = -u[p] * s + yq[q] * c;
                    double fx = X + cx, fy = Y + cy;
                    double i0 = floor(fx), j0 = floor(fy);
                    double ax = fx - i0, ay = fy - j0;
                    long i = (long)i0, j = (long)j0;
                    add_voxel(slice, nx, ny, i, j, (1.0 - ax) * (1.0 - ay) * g);
                    add_voxel(slice, nx, ny, i + 1, j, ax * (1.0 - ay) * g);
                    add_voxel(slice, nx, ny, i, j + 1, (1.0 - ax) * ay * g);
                    add_voxel(slice, nx, ny, i + 1, j + 1, ax * ay * g);
                }
            }
        }
    }
}
