/* Native IEEE single-precision evaluation of the float32 decision programs, used only to
 * pin the oracle's numpy emulation (every numpy float32 operation must round to float32).
 * Built by the test with gcc -O0 -ffp-contract=off on x86-64 (SSE arithmetic). */
#include <math.h>

void keys_cull(int n, const float *pts, const float *R, const float *t, float D, float zn,
               float gx, float gy, float *key, int *vis) {
  for (int i = 0; i < n; ++i) {
    float x = pts[3 * i], y = pts[3 * i + 1], z = pts[3 * i + 2];
    volatile float a, b, c;
    a = R[0] * x; b = R[1] * y; a = a + b; c = R[2] * z; a = a + c; float xc = a + t[0];
    a = R[3] * x; b = R[4] * y; a = a + b; c = R[5] * z; a = a + c; float yc = a + t[1];
    a = R[6] * x; b = R[7] * y; a = a + b; c = R[8] * z; a = a + c; float k = a + t[2];
    k = k + 0.0f;
    float zr = k - D;
    volatile float lx = gx * zr, ly = gy * zr;
    key[i] = k;
    vis[i] = isfinite(k) && isfinite(xc) && isfinite(yc) && zr > zn && fabsf(xc) <= lx && fabsf(yc) <= ly;
  }
}

void plane_coeffs(int K, const float *d, int V, const float *dx, float D, float inv_focal,
                  float ratio, float fp, float cp, float *b, float *C, float *Cn) {
  for (int k = 0; k < K; ++k) {
    volatile float z = d[k] - D;
    volatile float q = d[k] / z;
    volatile float m = d[k] * inv_focal;
    volatile float w = (1.0f - m) / z;
    b[k] = ratio * q;
    volatile float g = fp * w;
    for (int v = 0; v < V; ++v) {
      volatile float s = g * dx[v];
      volatile float c = cp + s;
      C[k * V + v] = c;
      Cn[k * V + v] = c + 0.5f;
    }
  }
}

void texel_coords(int n, const float *xs, float cx, float b, float C, float *X) {
  for (int i = 0; i < n; ++i) {
    volatile float xr = xs[i] - cx;
    volatile float p = b * xr;
    X[i] = p + C;
  }
}
