/*
 * FP64 CPU oracle for FDK cone-beam back-projection, after Chen et al.,
 * "iFDK: A Scalable Framework for Instant High-resolution Image
 * Reconstruction" (SC'19).
 *
 * TEST INFRASTRUCTURE ONLY. This is the plain, slow, obviously correct
 * reference the GPU library is checked against. Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it. The product
 * library never links, calls or falls back to it, and the two share no code,
 * header, table or constant.
 *
 * Every floating-point quantity is double precision. Loops follow the paper's
 * definitions directly: no blocking, no fusion, no reordering beyond what a
 * definition states. OpenMP only splits independent outputs across threads.
 *
 * Geometry vector g[14], one length unit throughout (Table 1):
 *   g[0..2]   Nx, Ny, Nz      voxel counts
 *   g[3..5]   Dx, Dy, Dz      voxel pitch
 *   g[6..7]   Nu, Nv          detector pixel counts
 *   g[8..9]   Du, Dv          detector pixel pitch
 *   g[10..11] off_u, off_v    principal-point shift in pixels (0 in the paper)
 *   g[12]     d               source to rotation axis
 *   g[13]     D               source to detector
 *
 * Arrays: volume V[k][j][i] is (Nz, Ny, Nx) with x fastest; projections
 * Q[s][v][u] are (Np, Nv, Nu) with u fastest.
 *
 * Readings taken where the paper is silent (each is listed in the design
 * notes): interp2 uses floor, not truncation; taps outside the detector read
 * zero; the principal point is ((Nu-1)/2 + off_u, (Nv-1)/2 + off_v); the ramp
 * convolution is linear (zero outside the row); the FDK constant pi*d^2/Np is
 * applied as a separate scale, not folded into the filter.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define G_NX(g) ((int64_t)(g)[0])
#define G_NY(g) ((int64_t)(g)[1])
#define G_NZ(g) ((int64_t)(g)[2])
#define G_NU(g) ((int64_t)(g)[6])
#define G_NV(g) ((int64_t)(g)[7])

int or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads later parallel loops use (for timing the oracle on one core). */
void or_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* ------------------------------------------------------------------ */
/* Geometry: Eq. (2), the projection matrix as the literal product      */
/* M1 * Mrot * M0 of 4x4 matrices, first three rows kept (3x4).         */
/* ------------------------------------------------------------------ */

static void mat4_mul(const double* A, const double* B, double* C) {
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) {
      double acc = 0.0;
      for (int m = 0; m < 4; ++m) acc += A[r * 4 + m] * B[m * 4 + c];
      C[r * 4 + c] = acc;
    }
}

/* M0: voxel index (i,j,k,1) -> world (X,Y,Z,1). Scale by the voxel pitch
 * after centring; j and k are negated (Eq. 2, M0). */
void or_m0(const double* g, double M0[16]) {
  const double S[16] = {g[3], 0, 0, 0, 0, g[4], 0, 0, 0, 0, g[5], 0, 0, 0, 0, 1};
  const double T[16] = {1, 0,  0,  -(g[0] - 1.0) / 2.0,
                        0, -1, 0,  (g[1] - 1.0) / 2.0,
                        0, 0,  -1, (g[2] - 1.0) / 2.0,
                        0, 0,  0,  1};
  mat4_mul(S, T, M0);
}

/* Full 4x4 projection P-hat = M1 * Mrot * M0 for gantry angle beta. */
void or_projection_matrix4(const double* g, double beta, double Ph[16]) {
  double M0[16], Mrot[16], M1[16], tmp[16];
  or_m0(g, M0);
  const double c = cos(beta), s = sin(beta), d = g[12], D = g[13];
  /* Mrot: rotation about Z by beta, then the axis swap and the shift by d. */
  const double A[16] = {1, 0, 0, 0, 0, 0, -1, 0, 0, 1, 0, d, 0, 0, 0, 1};
  const double R[16] = {c, -s, 0, 0, s, c, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1};
  mat4_mul(A, R, Mrot);
  /* M1: perspective onto the detector plane at distance D, principal point
   * at the detector centre (plus optional offsets), then pixel pitch. */
  const double cu = (g[6] - 1.0) / 2.0 + g[10], cv = (g[7] - 1.0) / 2.0 + g[11];
  const double S1[16] = {1.0 / g[8], 0, 0, 0, 0, 1.0 / g[9], 0, 0, 0, 0, 1, 0, 0, 0, 0, 1};
  const double K[16] = {D, 0, cu * g[8], 0, 0, D, cv * g[9], 0, 0, 0, 1, 0, 0, 0, 0, 1};
  mat4_mul(S1, K, M1);
  mat4_mul(Mrot, M0, tmp);
  mat4_mul(M1, tmp, Ph);
}

void or_projection_matrix(const double* g, double beta, double P[12]) {
  double Ph[16];
  or_projection_matrix4(g, beta, Ph);
  memcpy(P, Ph, 12 * sizeof(double));
}

/* ------------------------------------------------------------------ */
/* Counter-based input generator: SplitMix64 (Steele, Lea and Flood,    */
/* "Fast splittable pseudorandom number generators", OOPSLA 2014). The  */
/* value at counter c is the generator's output after c+1 state steps   */
/* from `seed`. Used only to regenerate synthetic inputs on demand.     */
/* ------------------------------------------------------------------ */

uint64_t or_splitmix64(uint64_t seed, uint64_t counter) {
  uint64_t z = seed + (counter + 1u) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* Uniform on [-1, 1) on the grid 2^-23: the top 24 output bits. */
double or_hash_uniform(uint64_t seed, uint64_t counter) {
  const int64_t m = (int64_t)(or_splitmix64(seed, counter) >> 40) - 8388608;
  return ldexp((double)m, -23);
}

/* Round to the nearest value with `sig` significant bits (ties to even),
 * with gradual underflow below 2^emin: the IEEE 754 rule for binary16
 * (sig 11, emin -14) and bfloat16 (sig 8, emin -126). No overflow handling:
 * generated inputs stay far below either format's maximum. */
static double round_sig(double x, int sig, int emin) {
  if (x == 0.0 || !isfinite(x)) return x;
  int e;
  frexp(x, &e); /* |x| = m * 2^e, m in [0.5, 1) -> leading bit weight 2^(e-1) */
  int lead = e - 1;
  if (lead < emin) lead = emin;
  const double quantum = ldexp(1.0, lead - (sig - 1));
  return nearbyint(x / quantum) * quantum;
}

double or_round_f16(double x) { return round_sig(x, 11, -14); }
double or_round_bf16(double x) { return round_sig(x, 8, -126); }

/* ------------------------------------------------------------------ */
/* Tap source for interp2: an explicit array Q, or generated values.    */
/* ------------------------------------------------------------------ */

typedef struct {
  const double* q; /* (np, nv, nu) or NULL for generated values */
  int64_t nu, nv;
  uint64_t seed;
  int rnd; /* generated values only: 0 none, 1 binary16, 2 bfloat16 */
} taps_t;

static double tap(const taps_t* t, int64_t s, int64_t a, int64_t b) {
  /* Reading: taps outside the detector read zero. */
  if (a < 0 || a >= t->nu || b < 0 || b >= t->nv) return 0.0;
  const int64_t idx = (s * t->nv + b) * t->nu + a;
  if (t->q) return t->q[idx];
  double x = or_hash_uniform(t->seed, (uint64_t)idx);
  if (t->rnd == 1) x = or_round_f16(x);
  if (t->rnd == 2) x = or_round_bf16(x);
  return x;
}

/* Alg. 3, bilinear interpolation X at sub-pixel (u, v); X(a, b) is
 * column a (u axis), row b (v axis). Reading: floor instead of int(). */
static double interp2(const taps_t* t, int64_t s, double u, double v) {
  const double fu = floor(u), fv = floor(v);
  const int64_t nu = (int64_t)fu, nv = (int64_t)fv;
  const double du = u - fu, dv = v - fv;
  const double t1 = tap(t, s, nu, nv) * (1.0 - du) + tap(t, s, nu + 1, nv) * du;
  const double t2 = tap(t, s, nu, nv + 1) * (1.0 - du) + tap(t, s, nu + 1, nv + 1) * du;
  return t1 * (1.0 - dv) + t2 * dv;
}

static double dot4(const double* row, double i, double j, double k) {
  return row[0] * i + row[1] * j + row[2] * k + row[3];
}

static double* all_matrices(const double* g, int64_t np, const double* angles) {
  double* P = (double*)malloc((size_t)np * 12 * sizeof(double));
  if (!P) return NULL;
  for (int64_t s = 0; s < np; ++s) or_projection_matrix(g, angles[s], P + 12 * s);
  return P;
}

/* One voxel of Alg. 2: sum over views of W_dis * interp2(Q_s, u, v) with
 * [x,y,z] = P_s [i,j,k,1], f = 1/z, W_dis = f^2, [u,v] = [x,y] f. */
static double alg2_voxel(const double* P, int64_t np, const taps_t* t,
                         int64_t i, int64_t j, int64_t k) {
  double acc = 0.0;
  for (int64_t s = 0; s < np; ++s) {
    const double* Ps = P + 12 * s;
    const double x = dot4(Ps + 0, (double)i, (double)j, (double)k);
    const double y = dot4(Ps + 4, (double)i, (double)j, (double)k);
    const double z = dot4(Ps + 8, (double)i, (double)j, (double)k);
    const double f = 1.0 / z;
    const double W = f * f;
    acc += W * interp2(t, s, x * f, y * f);
  }
  return acc;
}

/* Back-projection, Alg. 2, FP64.
 *   q      (np, nv, nu) doubles, or NULL to generate taps from `seed`
 *          (rnd: 0 as generated, 1 rounded to binary16, 2 to bfloat16)
 *   ijk    NULL: every voxel, out is (Nz, Ny, Nx)
 *          else: nvox triples (i, j, k) of global voxel indices, out[nvox]
 * out = scale * sum_s W_dis * interp2(Q_s, u, v). Returns 0, or -1 on
 * allocation failure. */
int or_backproject(const double* g, int64_t np, const double* angles,
                   const double* q, uint64_t seed, int rnd, double scale,
                   int64_t nvox, const int64_t* ijk, double* out) {
  double* P = all_matrices(g, np, angles);
  if (!P) return -1;
  const taps_t t = {q, G_NU(g), G_NV(g), seed, rnd};
  const int64_t nx = G_NX(g), ny = G_NY(g), nz = G_NZ(g);
  const int64_t n = ijk ? nvox : nx * ny * nz;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t m = 0; m < n; ++m) {
    int64_t i, j, k;
    if (ijk) {
      i = ijk[3 * m];
      j = ijk[3 * m + 1];
      k = ijk[3 * m + 2];
    } else {
      i = m % nx;
      j = (m / nx) % ny;
      k = m / (nx * ny);
    }
    out[m] = scale * alg2_voxel(P, np, &t, i, j, k);
  }
  free(P);
  return 0;
}

/* Back-projection, Alg. 4 (the paper's reduced-cost form), written
 * independently of Alg. 2 so each pins the other. Per view and column:
 * x and z from two inner products at k = 0 (Theorems 2, 3), f, u, W once;
 * per k below the mid-plane one inner product for y, v = y f; the mirrored
 * voxel Nz-1-k takes v~ = 2 c_v - v (Theorem 1, with c_v the principal row;
 * this is Nv-1-v when off_v = 0). An odd middle slice is done once,
 * unmirrored. Full volume only; explicit array Q only. */
int or_backproject_alg4(const double* g, int64_t np, const double* angles,
                        const double* q, double scale, double* out) {
  const int64_t nx = G_NX(g), ny = G_NY(g), nz = G_NZ(g);
  const double cv2 = (g[7] - 1.0) + 2.0 * g[11];
  const taps_t t = {q, G_NU(g), G_NV(g), 0, 0};
  memset(out, 0, (size_t)(nx * ny * nz) * sizeof(double));
  double Ps[12];
  for (int64_t s = 0; s < np; ++s) {
    or_projection_matrix(g, angles[s], Ps);
#pragma omp parallel for schedule(static)
    for (int64_t col = 0; col < nx * ny; ++col) {
      const int64_t i = col % nx, j = col / nx;
      const double x = dot4(Ps + 0, (double)i, (double)j, 0.0);
      const double z = dot4(Ps + 8, (double)i, (double)j, 0.0);
      const double f = 1.0 / z;
      const double u = x * f;
      const double W = f * f;
      for (int64_t k = 0; k < nz / 2; ++k) {
        const double y = dot4(Ps + 4, (double)i, (double)j, (double)k);
        const double v = y * f;
        out[(k * ny + j) * nx + i] += W * interp2(&t, s, u, v);
        const int64_t kt = nz - 1 - k;
        const double vt = cv2 - v;
        out[(kt * ny + j) * nx + i] += W * interp2(&t, s, u, vt);
      }
      if (nz % 2) {
        const int64_t k = nz / 2;
        const double v = dot4(Ps + 4, (double)i, (double)j, (double)k) * f;
        out[(k * ny + j) * nx + i] += W * interp2(&t, s, u, v);
      }
    }
  }
  for (int64_t m = 0; m < nx * ny * nz; ++m) out[m] *= scale;
  return 0;
}

/* Forward projection: the exact transpose (adjoint) of or_backproject over
 * the full volume. Every voxel, for every view, adds scale * W_dis * (its
 * bilinear weight) * V[k][j][i] into each of its four taps that lies inside
 * the detector. out is (np, nv, nu), overwritten. Parallel over views, so
 * no two threads touch the same output. */
int or_forward_project(const double* g, int64_t np, const double* angles,
                       const double* vol, double scale, double* out) {
  double* P = all_matrices(g, np, angles);
  if (!P) return -1;
  const int64_t nx = G_NX(g), ny = G_NY(g), nz = G_NZ(g);
  const int64_t nu = G_NU(g), nv = G_NV(g);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t s = 0; s < np; ++s) {
    const double* Ps = P + 12 * s;
    double* qs = out + s * nu * nv;
    memset(qs, 0, (size_t)(nu * nv) * sizeof(double));
    for (int64_t k = 0; k < nz; ++k)
      for (int64_t j = 0; j < ny; ++j)
        for (int64_t i = 0; i < nx; ++i) {
          const double val = vol[(k * ny + j) * nx + i];
          const double x = dot4(Ps + 0, (double)i, (double)j, (double)k);
          const double y = dot4(Ps + 4, (double)i, (double)j, (double)k);
          const double z = dot4(Ps + 8, (double)i, (double)j, (double)k);
          const double f = 1.0 / z;
          const double W = f * f;
          const double u = x * f, v = y * f;
          const double fu = floor(u), fv = floor(v);
          const int64_t a0 = (int64_t)fu, b0 = (int64_t)fv;
          const double du = u - fu, dv = v - fv;
          const double wt[2][2] = {{(1.0 - du) * (1.0 - dv), du * (1.0 - dv)},
                                   {(1.0 - du) * dv, du * dv}};
          for (int bb = 0; bb < 2; ++bb)
            for (int aa = 0; aa < 2; ++aa) {
              const int64_t a = a0 + aa, b = b0 + bb;
              if (a < 0 || a >= nu || b < 0 || b >= nv) continue;
              qs[b * nu + a] += scale * W * wt[bb][aa] * val;
            }
        }
  }
  free(P);
  return 0;
}

/* ------------------------------------------------------------------ */
/* Phantom: analytic line integrals through a sum of ellipsoids.        */
/* ------------------------------------------------------------------ */

/* Source and detector-pixel positions in world coordinates, obtained by
 * inverting Eq. (2): Mrot*M0 maps world (X,Y,Z) to gantry coordinates
 * (a, b, c) = (cos*X - sin*Y, -Z, sin*X + cos*Y + d); M1 then gives
 * u = D a / (Du c) + c_u and v = D b / (Dv c) + c_v. The source is the
 * gantry origin (z = c = 0); pixel (u, v) sits on the plane c = D at
 * a = (u - c_u) Du, b = (v - c_v) Dv. */
void or_source_pixel(const double* g, double beta, double u, double v,
                     double src[3], double pix[3]) {
  const double c = cos(beta), s = sin(beta), d = g[12], D = g[13];
  const double cu = (g[6] - 1.0) / 2.0 + g[10], cv = (g[7] - 1.0) / 2.0 + g[11];
  src[0] = -d * s;
  src[1] = -d * c;
  src[2] = 0.0;
  const double a = (u - cu) * g[8], b = (v - cv) * g[9];
  const double Xr = a, Yr = D - d, Zr = -b; /* rotated world coordinates */
  pix[0] = c * Xr + s * Yr;
  pix[1] = -s * Xr + c * Yr;
  pix[2] = Zr;
}

/* Ellipsoid record, 16 doubles: centre (3), semi-axes (3), rotation R
 * (3x3 row-major; its columns are the ellipsoid's axes in world
 * coordinates), density. A point p is inside when
 * sum_m ((R^T (p - c))_m / a_m)^2 <= 1. Densities of overlaps add. */
static void to_unit_frame(const double* e, const double p[3], int is_dir, double o[3]) {
  const double* R = e + 6;
  double w[3];
  for (int m = 0; m < 3; ++m) w[m] = is_dir ? p[m] : p[m] - e[m];
  for (int m = 0; m < 3; ++m)
    o[m] = (R[0 * 3 + m] * w[0] + R[1 * 3 + m] * w[1] + R[2 * 3 + m] * w[2]) / e[3 + m];
}

/* Integral of the density along the whole line src + t * dir. */
double or_ray_integral(const double src[3], const double dir[3], int64_t nell,
                       const double* ell) {
  const double len = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
  double acc = 0.0;
  for (int64_t n = 0; n < nell; ++n) {
    const double* e = ell + 16 * n;
    double o[3], w[3];
    to_unit_frame(e, src, 0, o);
    to_unit_frame(e, dir, 1, w);
    const double A = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    const double B = o[0] * w[0] + o[1] * w[1] + o[2] * w[2];
    const double C = o[0] * o[0] + o[1] * o[1] + o[2] * o[2] - 1.0;
    const double disc = B * B - A * C;
    if (disc > 0.0) acc += e[15] * (2.0 * sqrt(disc) / A) * len;
  }
  return acc;
}

/* Line integrals E (np, nv, nu) of the phantom for every detector pixel
 * centre of every view. */
void or_phantom_project(const double* g, int64_t np, const double* angles,
                        int64_t nell, const double* ell, double* out) {
  const int64_t nu = G_NU(g), nv = G_NV(g);
#pragma omp parallel for collapse(2) schedule(dynamic, 4)
  for (int64_t s = 0; s < np; ++s)
    for (int64_t b = 0; b < nv; ++b) {
      for (int64_t a = 0; a < nu; ++a) {
        double src[3], pix[3], dir[3];
        or_source_pixel(g, angles[s], (double)a, (double)b, src, pix);
        for (int m = 0; m < 3; ++m) dir[m] = pix[m] - src[m];
        out[(s * nv + b) * nu + a] = or_ray_integral(src, dir, nell, ell);
      }
    }
}

/* Line integrals for a list of (view, row, column) pixels. */
void or_phantom_project_pixels(const double* g, const double* angles,
                               int64_t npix, const int64_t* svu, int64_t nell,
                               const double* ell, double* out) {
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t m = 0; m < npix; ++m) {
    double src[3], pix[3], dir[3];
    or_source_pixel(g, angles[svu[3 * m]], (double)svu[3 * m + 2],
                    (double)svu[3 * m + 1], src, pix);
    for (int c = 0; c < 3; ++c) dir[c] = pix[c] - src[c];
    out[m] = or_ray_integral(src, dir, nell, ell);
  }
}

/* Density of the phantom at world points pts (npts, 3). */
void or_phantom_density(int64_t nell, const double* ell, int64_t npts,
                        const double* pts, double* out) {
#pragma omp parallel for schedule(static)
  for (int64_t m = 0; m < npts; ++m) {
    double acc = 0.0;
    for (int64_t n = 0; n < nell; ++n) {
      double o[3];
      to_unit_frame(ell + 16 * n, pts + 3 * m, 0, o);
      if (o[0] * o[0] + o[1] * o[1] + o[2] * o[2] <= 1.0) acc += ell[16 * n + 15];
    }
    out[m] = acc;
  }
}

/* ------------------------------------------------------------------ */
/* Filtering stage, Alg. 1: cosine weighting, then a ramp convolution   */
/* along each detector row.                                             */
/* ------------------------------------------------------------------ */

/* Discrete ramp kernel h(n) sampled at pitch tau (the detector pitch
 * scaled to the rotation axis). kind 0: Ram-Lak, kind 1: Shepp-Logan. */
double or_ramp_kernel(int kind, int64_t n, double tau) {
  const double pi = 3.14159265358979323846;
  if (kind == 0) {
    if (n == 0) return 1.0 / (4.0 * tau * tau);
    if (n % 2 == 0) return 0.0;
    return -1.0 / ((double)n * (double)n * pi * pi * tau * tau);
  }
  return -2.0 / (pi * pi * tau * tau * (4.0 * (double)n * (double)n - 1.0));
}

/* Cosine weight: D / sqrt(D^2 + a^2 + b^2) with (a, b) the pixel's
 * distance from the principal point on the detector. */
double or_cos_weight(const double* g, double u, double v) {
  const double cu = (g[6] - 1.0) / 2.0 + g[10], cv = (g[7] - 1.0) / 2.0 + g[11];
  const double a = (u - cu) * g[8], b = (v - cv) * g[9], D = g[13];
  return D / sqrt(D * D + a * a + b * b);
}

/* Alg. 1 for one detector row b: E~ = E * F_cos point-wise, then
 * Q(u) = tau * sum_n h(u - n) E~(n), a direct linear convolution (zero
 * outside the row). h holds h(n) for n in [-nu, nu] at h[n + nu]; et is
 * nu doubles of scratch. */
static void filter_row(const double* g, const double* h, double tau, int64_t b,
                       const double* row, double* et, double* qrow) {
  const int64_t nu = G_NU(g);
  for (int64_t n = 0; n < nu; ++n) et[n] = row[n] * or_cos_weight(g, (double)n, (double)b);
  for (int64_t a = 0; a < nu; ++a) {
    double acc = 0.0;
    for (int64_t n = 0; n < nu; ++n) acc += h[a - n + nu] * et[n];
    qrow[a] = tau * acc;
  }
}

/* Alg. 1 on nrows rows of nu values; row m is detector row rows_v[m]
 * (its cosine weights depend on it). e and out are (nrows, nu). Returns -1
 * on allocation failure. */
int or_filter_rows(const double* g, int64_t nrows, const int64_t* rows_v, int kind,
                   const double* e, double* out) {
  const int64_t nu = G_NU(g);
  const double tau = g[8] * g[12] / g[13];
  double* h = (double*)malloc((size_t)(2 * nu + 1) * sizeof(double));
  if (!h) return -1;
  for (int64_t n = -nu; n <= nu; ++n) h[n + nu] = or_ramp_kernel(kind, n, tau);
  int failed = 0;
#pragma omp parallel
  {
    double* et = (double*)malloc((size_t)nu * sizeof(double));
    if (!et) {
#pragma omp atomic write
      failed = 1;
    }
#pragma omp for schedule(static)
    for (int64_t m = 0; m < nrows; ++m) {
      if (!et) continue;
      filter_row(g, h, tau, rows_v[m], e + m * nu, et, out + m * nu);
    }
    free(et);
  }
  free(h);
  return failed ? -1 : 0;
}

/* Transpose of Alg. 1 on whole views: for the operator
 * Q(b, a) = tau * sum_n h(a - n) * F_cos(n, b) * E(b, n), the transpose maps G
 * to E_grad(b, n) = F_cos(n, b) * tau * sum_a h(a - n) * G(b, a), the sum over
 * the forward operator's output index written out as such. g and out are
 * (nviews, nv, nu). Returns -1 on allocation failure. */
int or_filter_adjoint(const double* g, int64_t nviews, int kind, const double* gq, double* out) {
  const int64_t nu = G_NU(g), nv = G_NV(g);
  const double tau = g[8] * g[12] / g[13];
  double* h = (double*)malloc((size_t)(2 * nu + 1) * sizeof(double));
  if (!h) return -1;
  for (int64_t n = -nu; n <= nu; ++n) h[n + nu] = or_ramp_kernel(kind, n, tau);
#pragma omp parallel for collapse(2) schedule(static)
  for (int64_t s = 0; s < nviews; ++s)
    for (int64_t b = 0; b < nv; ++b) {
      const double* grow = gq + (s * nv + b) * nu;
      double* erow = out + (s * nv + b) * nu;
      for (int64_t n = 0; n < nu; ++n) {
        double acc = 0.0;
        for (int64_t a = 0; a < nu; ++a) acc += h[a - n + nu] * grow[a];
        erow[n] = or_cos_weight(g, (double)n, (double)b) * tau * acc;
      }
    }
  free(h);
  return 0;
}

/* Alg. 1 on whole views: e and out are (nviews, nv, nu). */
int or_filter(const double* g, int64_t nviews, int kind, const double* e, double* out) {
  const int64_t nv = G_NV(g);
  int64_t* rows_v = (int64_t*)malloc((size_t)(nviews * nv) * sizeof(int64_t));
  if (!rows_v) return -1;
  for (int64_t m = 0; m < nviews * nv; ++m) rows_v[m] = m % nv;
  const int rc = or_filter_rows(g, nviews * nv, rows_v, kind, e, out);
  free(rows_v);
  return rc;
}

/* Generated tap values for a list of counters (for tests of the
 * generator itself and for building inputs on the host). */
void or_hash_fill(uint64_t seed, int64_t n, const uint64_t* counters, int rnd, double* out) {
  for (int64_t m = 0; m < n; ++m) {
    double x = or_hash_uniform(seed, counters[m]);
    if (rnd == 1) x = or_round_f16(x);
    if (rnd == 2) x = or_round_bf16(x);
    out[m] = x;
  }
}
