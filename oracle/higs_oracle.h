/*
 * Types shared by the two files of the FP64 CPU oracle (the forward path in
 * higs_oracle.c, its adjoint in higs_oracle_grad.c).  TEST INFRASTRUCTURE
 * ONLY: nothing outside oracle/ includes this header.
 */
#ifndef HIGS_ORACLE_H
#define HIGS_ORACLE_H
#include <stdint.h>

#define OC_TILE 8          /* render tile edge, pixels (sec. 3.1) */
#define OC_MT_TX 8         /* macro-tile width in render tiles */
#define OC_MT_TY 4         /* macro-tile height in render tiles */
#define OC_MT_W (OC_TILE * OC_MT_TX) /* 64 px */
#define OC_MT_H (OC_TILE * OC_MT_TY) /* 32 px */

/* Columns of the per-gaussian double record written by oc_project. */
enum {
  G_TZ = 0, G_MX, G_MY, G_A, G_B, G_C, G_TAU, G_L0, G_L1, G_L2, G_OP,
  G_R, G_G, G_BL, G_NCOL
};

typedef struct {
  int32_t width, height;
  float fx, fy, cx, cy;
  float world_to_cam[12]; /* row-major [R | t], x_cam = R x_world + t */
  float background[3];
} oc_camera;

typedef struct {
  double near_z;     /* cull when camera-space z <= near_z */
  double alpha_min;  /* skip contributions with alpha below it; the opacity
                        level tau assumes the paper's 1/255 */
  double alpha_max;  /* 0.99 clamp on alpha */
  double t_eps;      /* stop once transmittance < t_eps (after compositing) */
  double dilation;   /* added to the diagonal of the 2D covariance */
  int32_t batch_cap; /* B_r */
  int32_t sh_degree; /* 0..3 */
} oc_params;

/* Flags for a pixel whose GPU result may legitimately differ from the
 * oracle by more than rounding: a contribution decided at alpha ~ alpha_min,
 * or a transmittance landing next to t_eps. */
#define OC_AMB_ALPHA 1
#define OC_AMB_T 2

void oc_sh_basis(const double d[3], int degree, double out[16]);
double oc_f32_q_bound(const double* rec, double dx, double dy, double u, double v, double q);
uint32_t oc_depth_key(double tz);

#endif
