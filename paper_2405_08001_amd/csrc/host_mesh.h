// Host-side mesh preprocessing shared by the single-scene context and the
// batch: rest-shape inverses and the wave-packed vertex incidence.
#pragma once

#include <algorithm>
#include <vector>

#include "internal.h"

namespace pncg {

// D_m = [X1-X0, X2-X0, X3-X0]; Bm[e] = rows of D_m^{-1} (9 values), vol[e] =
// det(D_m) / 6.  Returns the index of the first tet with det <= 0, or -1.
inline int rest_shape(const double* X, const int* tets, int nT, std::vector<double>& Bm, std::vector<double>& vol) {
  Bm.assign(9 * (size_t)nT, 0.0);
  vol.assign(nT, 0.0);
  for (int e = 0; e < nT; ++e) {
    const int* t = tets + 4 * e;
    double D[3][3];
    for (int j = 0; j < 3; ++j)
      for (int i = 0; i < 3; ++i) D[i][j] = X[3 * t[j + 1] + i] - X[3 * t[0] + i];
    const double det = D[0][0] * (D[1][1] * D[2][2] - D[1][2] * D[2][1]) -
                       D[0][1] * (D[1][0] * D[2][2] - D[1][2] * D[2][0]) +
                       D[0][2] * (D[1][0] * D[2][1] - D[1][1] * D[2][0]);
    if (!(det > 0.0)) return e;
    const double id = 1.0 / det;
    double Inv[3][3];
    Inv[0][0] = (D[1][1] * D[2][2] - D[1][2] * D[2][1]) * id;
    Inv[0][1] = (D[0][2] * D[2][1] - D[0][1] * D[2][2]) * id;
    Inv[0][2] = (D[0][1] * D[1][2] - D[0][2] * D[1][1]) * id;
    Inv[1][0] = (D[1][2] * D[2][0] - D[1][0] * D[2][2]) * id;
    Inv[1][1] = (D[0][0] * D[2][2] - D[0][2] * D[2][0]) * id;
    Inv[1][2] = (D[0][2] * D[1][0] - D[0][0] * D[1][2]) * id;
    Inv[2][0] = (D[1][0] * D[2][1] - D[1][1] * D[2][0]) * id;
    Inv[2][1] = (D[0][1] * D[2][0] - D[0][0] * D[2][1]) * id;
    Inv[2][2] = (D[0][0] * D[1][1] - D[0][1] * D[1][0]) * id;
    for (int r = 0; r < 3; ++r)
      for (int j = 0; j < 3; ++j) Bm[9 * (size_t)e + 3 * r + j] = Inv[r][j];
    vol[e] = det / 6.0;
  }
  return -1;
}

// Vertex -> (tet, corner) incidence as lanes (tet * 4 + corner, vertex),
// grouped by vertex, the tets of a vertex in increasing order, packed into
// 64-lane waves without splitting a vertex across waves; a vertex without
// tets gets one lane with code -2.  `tets` holds local indices; `tet_base`
// and `vert_base` are added to the stored tet and vertex ids.  Appends to
// inc / incv; false if a vertex has more than 64 tets.
inline bool pack_incidence(int nV, const int* tets, int nT, int vert_base, std::vector<int>& inc,
                           std::vector<int>& incv, int tet_base = 0) {
  std::vector<int> deg(nV, 0);
  for (long long i = 0; i < 4LL * nT; ++i) deg[tets[i]]++;
  for (int v = 0; v < nV; ++v)
    if (deg[v] > kWave) return false;
  std::vector<int> off(nV + 1, 0);
  for (int v = 0; v < nV; ++v) off[v + 1] = off[v] + deg[v];
  std::vector<int> lst(4 * (size_t)nT), fill(off.begin(), off.end() - 1);
  for (int e = 0; e < nT; ++e)
    for (int a = 0; a < 4; ++a) lst[fill[tets[4 * e + a]]++] = 4 * (e + tet_base) + a;
  int used = 0;
  for (int v = 0; v < nV; ++v) {
    const int d = std::max(deg[v], 1);
    if (used + d > kWave) {
      while (used < kWave) { inc.push_back(-1); incv.push_back(-1); ++used; }
      used = 0;
    }
    if (deg[v] == 0) { inc.push_back(-2); incv.push_back(v + vert_base); }
    for (int i = off[v]; i < off[v + 1]; ++i) { inc.push_back(lst[i]); incv.push_back(v + vert_base); }
    used += d;
  }
  while (used % kWave) { inc.push_back(-1); incv.push_back(-1); ++used; }
  return true;
}

}  // namespace pncg
