/*
 * Synthetic pencil-beam dose-influence generator (input synthesis only).
 *
 * Builds, for one uncertainty scenario, the nonnegative dose-influence matrix
 * A (voxels x spots) whose entry A[i,j] is the dose deposited in voxel i by
 * spot j at unit intensity (the A_s of the problem statement, Sec. 2.1).  The
 * paper computes these with a clinical pencil-beam engine on CT images; this
 * file stands in for that engine with an analytic model:
 *
 *   A[i,j] = exp(-r^2 / (2 sigma^2)) * bragg(depth; R_j)
 *
 * where r is the lateral distance of voxel i from the central axis of spot j,
 * depth is the distance along that axis from the point where it enters the
 * body, and bragg() is a Bragg-like depth profile (entrance plateau rising to a
 * unit peak at the range R_j, then a Gaussian distal fall-off).  Entries below
 * drop_rel times the column maximum are dropped, and values are rounded to
 * float32 so every consumer sees exactly the same matrix.
 *
 * Nothing here solves or evaluates the optimisation problem: this module only
 * produces its inputs, in CSR form (rows sorted, columns ascending within a
 * row).  The result is independent of the number of OpenMP threads.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int64_t nnz;
  int32_t m, n;
  int64_t* row_ptr; /* m+1 */
  int32_t* col;     /* nnz */
  float* val;       /* nnz */
} synth_csr;

typedef struct {
  int32_t cap, len;
  int32_t* row;
  float* val;
} spot_list;

static int spot_push(spot_list* s, int32_t row, float v) {
  if (s->len == s->cap) {
    int32_t nc = s->cap ? 2 * s->cap : 1024;
    int32_t* nr = (int32_t*)realloc(s->row, (size_t)nc * sizeof(int32_t));
    if (!nr) return -1;
    s->row = nr;
    float* nv = (float*)realloc(s->val, (size_t)nc * sizeof(float));
    if (!nv) return -1;
    s->val = nv;
    s->cap = nc;
  }
  s->row[s->len] = row;
  s->val[s->len] = v;
  s->len++;
  return 0;
}

/* Bragg-like depth profile with unit peak at depth R (mm). */
static double bragg(double d, double R) {
  if (d < 0.0) d = 0.0;
  if (d <= R) {
    double f = d / R;
    double plateau = 0.3 + 0.2 * f;
    double wp = 0.04 * R + 1.0;
    double e = (R - d) / wp;
    return plateau + 0.5 * exp(-0.5 * e * e);
  }
  double wd = 0.012 * R + 0.8;
  double e = (d - R) / wd;
  return exp(-0.5 * e * e);
}

static double distal_extent(double R) { return R + 5.0 * (0.012 * R + 0.8); }

/*
 * Generate one scenario.
 *   grid nx*ny*nz, voxel size h (mm); voxel centre ((ix+.5)h, (iy+.5)h, (iz+.5)h);
 *   linear voxel index = ix + nx*(iy + ny*iz);
 *   row_of_voxel[v] = matrix row of voxel v, or -1 when the voxel is not a row.
 *   spot j: origin[3j..] = entry point of its central axis into the body (mm),
 *           axis[3j..] = unit direction of travel, range[j] = R_j (mm).
 * Returns 0 on success, -1 on allocation failure, -2 on bad arguments.
 */
int synth_dose_csr(int32_t nx, int32_t ny, int32_t nz, double h,
                   const int32_t* row_of_voxel, int32_t m, int32_t n,
                   const double* origin, const double* axis,
                   const double* range, double sigma, double drop_rel,
                   synth_csr* out) {
  if (!out || nx <= 0 || ny <= 0 || nz <= 0 || h <= 0 || m < 0 || n < 0 ||
      sigma <= 0 || drop_rel <= 0 || drop_rel >= 1)
    return -2;
  memset(out, 0, sizeof(*out));
  out->m = m;
  out->n = n;
  spot_list* lists = (spot_list*)calloc((size_t)(n > 0 ? n : 1), sizeof(spot_list));
  if (!lists) return -1;
  const double rmax = sigma * sqrt(2.0 * log(1.0 / drop_rel));
  int failed = 0;

#pragma omp parallel for schedule(dynamic, 4) reduction(| : failed)
  for (int32_t j = 0; j < n; ++j) {
    const double* o = origin + 3 * (size_t)j;
    const double* a = axis + 3 * (size_t)j;
    const double R = range[j];
    const double L = distal_extent(R);
    double lo[3], hi[3];
    for (int k = 0; k < 3; ++k) {
      double e0 = o[k], e1 = o[k] + L * a[k];
      double mn = e0 < e1 ? e0 : e1, mx = e0 < e1 ? e1 : e0;
      /* the disc of radius rmax around the axis spans at most rmax*sqrt(1-a_k^2) */
      double ext = rmax * sqrt(fmax(0.0, 1.0 - a[k] * a[k]));
      lo[k] = mn - ext;
      hi[k] = mx + ext;
    }
    int32_t ilo[3], ihi[3];
    const int32_t dims[3] = {nx, ny, nz};
    for (int k = 0; k < 3; ++k) {
      int32_t l = (int32_t)floor(lo[k] / h - 0.5);
      int32_t u = (int32_t)ceil(hi[k] / h - 0.5);
      ilo[k] = l < 0 ? 0 : l;
      ihi[k] = u > dims[k] - 1 ? dims[k] - 1 : u;
    }
    spot_list* s = &lists[j];
    double colmax = 0.0;
    for (int32_t iz = ilo[2]; iz <= ihi[2]; ++iz) {
      double cz = (iz + 0.5) * h - o[2];
      for (int32_t iy = ilo[1]; iy <= ihi[1]; ++iy) {
        double cy = (iy + 0.5) * h - o[1];
        for (int32_t ix = ilo[0]; ix <= ihi[0]; ++ix) {
          int64_t vox = ix + (int64_t)nx * (iy + (int64_t)ny * iz);
          int32_t row = row_of_voxel[vox];
          if (row < 0) continue;
          double cx = (ix + 0.5) * h - o[0];
          double t = cx * a[0] + cy * a[1] + cz * a[2];
          if (t > L) continue;
          double r2 = cx * cx + cy * cy + cz * cz - t * t;
          if (r2 < 0) r2 = 0;
          if (r2 > rmax * rmax) continue;
          double v = exp(-0.5 * r2 / (sigma * sigma)) * bragg(t, R);
          if (v > colmax) colmax = v;
          if (spot_push(s, row, (float)v)) failed |= 1;
        }
      }
    }
    /* drop entries below drop_rel * column maximum, in place */
    const double thr = drop_rel * colmax;
    int32_t w = 0;
    for (int32_t k = 0; k < s->len; ++k) {
      if ((double)s->val[k] >= thr && s->val[k] > 0.0f) {
        s->row[w] = s->row[k];
        s->val[w] = s->val[k];
        ++w;
      }
    }
    s->len = w;
  }

  int rc = failed ? -1 : 0;
  if (!rc) {
    int64_t nnz = 0;
    for (int32_t j = 0; j < n; ++j) nnz += lists[j].len;
    out->nnz = nnz;
    out->row_ptr = (int64_t*)calloc((size_t)m + 1, sizeof(int64_t));
    out->col = (int32_t*)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));
    out->val = (float*)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(float));
    if (!out->row_ptr || !out->col || !out->val) {
      rc = -1;
    } else {
      /* counting sort by row; visiting spots in increasing j keeps columns sorted */
      for (int32_t j = 0; j < n; ++j)
        for (int32_t k = 0; k < lists[j].len; ++k) out->row_ptr[lists[j].row[k] + 1]++;
      for (int32_t i = 0; i < m; ++i) out->row_ptr[i + 1] += out->row_ptr[i];
      int64_t* cursor = (int64_t*)malloc((size_t)(m > 0 ? m : 1) * sizeof(int64_t));
      if (!cursor) {
        rc = -1;
      } else {
        memcpy(cursor, out->row_ptr, (size_t)m * sizeof(int64_t));
        for (int32_t j = 0; j < n; ++j)
          for (int32_t k = 0; k < lists[j].len; ++k) {
            int64_t p = cursor[lists[j].row[k]]++;
            out->col[p] = j;
            out->val[p] = lists[j].val[k];
          }
        free(cursor);
      }
    }
  }
  for (int32_t j = 0; j < n; ++j) {
    free(lists[j].row);
    free(lists[j].val);
  }
  free(lists);
  if (rc) {
    free(out->row_ptr);
    free(out->col);
    free(out->val);
    memset(out, 0, sizeof(*out));
  }
  return rc;
}

void synth_csr_free(synth_csr* c) {
  if (!c) return;
  free(c->row_ptr);
  free(c->col);
  free(c->val);
  memset(c, 0, sizeof(*c));
}
