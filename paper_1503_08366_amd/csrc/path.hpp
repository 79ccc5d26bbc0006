// Lambda-path iteration (R problems sharing one scaled matrix and factor).
#pragma once

#include "internal.hpp"

namespace pogs {

struct PathArgs {
  int m, n, ld, q, ldk;
  int R, Rp;               // problems, padded to a multiple of 64 (state matrices have Rp columns)
  int nbx, nby;            // prox row blocks over n and m
  int nb_pri, nb_dual;     // reduce row blocks over m and n
  int rows_per_block;
  float alpha;
  double delta, tau, eps_abs, eps_rel;
  int max_iter, adaptive;
  const float *A, *Kinv;
  const uint8_t *fh, *gh;                   // m x Rp, n x Rp
  const float *fa, *fb, *fc, *fd, *fe;      // m x Rp each
  const float *ga, *gb, *gc, *gd, *ge;      // n x Rp each
  float *XX;                                // n x 2Rp: [X | Xh]
  float *Xt, *Mu, *Cx;                      // n x Rp
  float *DN;                                // m x 2Rp: [Dy | Nu]
  float *Y, *Yt, *Yh;                       // m x Rp
  float *Rhs;                               // n x Rp
  double *s_mu, *s_yh, *s_pri, *s_dual;     // [blocks][Rp] partial sums
  double *rho, *rescale, *r_pri, *r_dual, *eps_pri, *eps_dual;  // per problem
  int *l, *u, *iters, *done, *status;       // per problem
  int *all_done;
};

void path_geometry(PathArgs *p, int *s1, int *s2, int *s3);
size_t path_part_floats(int m, int n, int Rp);
void launch_path_scale_fn(const double *src, const uint8_t *hsrc, int len, int Rp, const double *scale, bool divide,
                          uint8_t *h, float *a, float *b, float *c, float *d, float *e, hipStream_t s);
void launch_path_iteration(const PathArgs &p, float *part, hipStream_t s);
void launch_path_unscale(const PathArgs &p, const double *D, const double *E, const double *f0, const uint8_t *fh0,
                         const double *g0, const uint8_t *gh0, float *out, double *obj, hipStream_t s);

}  // namespace pogs
