// Kernels of the Green's-function build (Sec. 2, Eq. (green_mat)); see green_kernels.hip.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

// X[k][i][n'] = c_{i, n0+n'}(k) w, w = e^{-(mu - eps) tau} (occupied = 1) or e^{-(eps - mu) tau};
// eps [nk][nb], wfc complex [nk][nb][nb] (c_{in}(k) at [k][i][n]), X complex [nk][nb][nbs].
hipError_t launch_green_weight(const double *eps, const double *wfc, int nk, int nb, int n0, int nbs, double mu,
                               double tau, int occupied, double *X, hipStream_t s);
// G[R][e] = Re sum_k ph[R][k] W[k][e] for e < m; ph device complex [nR][nk] (2 nR nk doubles,
// at most 64 KiB), W complex [nk][m], G real [nR][m].
hipError_t launch_k2r_real(const double *ph, int nR, int nk, size_t m, const double *W, double *G, hipStream_t s);
// out[0] = max |G^s(-R)_{ji} - G^s(R)_{ij}|, out[1] = max |G^s(R)_{ij}| over s, tau, R, i, j for
// G_occ, G_un [ntau][nR][nb][nb] on the BvK mesh (out: 2 device doubles, cleared by the launcher).
hipError_t launch_green_symmetry(const double *Gocc, const double *Gun, int ntau, const int mesh[3], int nb,
                                 double *out, hipStream_t s);
