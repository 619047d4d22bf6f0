// Host assembly of the P1 finite-element quantities of one island mesh.
//
// For each tetrahedron e with vertices p0..p3 the barycentric gradients come from the inverse of
// the 3x3 matrix J whose rows are the edge vectors p1-p0, p2-p0, p3-p0: grad(phi_a) for a = 1..3
// is column a-1 of J^-1 and grad(phi_0) = -(sum of the others).  From them:
//   V_i      = sum_e V_e / 4                          lumped node volume
//   K_ij     = sum_e V_e grad(phi_i) . grad(phi_j)     exchange stiffness (E_ex = A m^T K m)
//   D_k,(j,a)= sum_e (V_e / 4) d_a phi_k |_e           charge of node k: b_k = int M . grad phi_k
//   a_i      = lumped area of node i on the soft/hard interface (faces with three interface
//              nodes of one layer, one third of the face area per node)
// The paper's island (Sec. II.B, Fig. 3) has a soft and a hard layer joined by an interlayer
// exchange; the two layers are meshed separately and the interface nodes are paired.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "bpm_internal.h"

namespace bpm {

static bool invert3(const double J[3][3], double Ji[3][3], double* det_out) {
  double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
  double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
  if (!(std::fabs(det) > 0.0)) return false;
  double id = 1.0 / det;
  Ji[0][0] = c00 * id;
  Ji[1][0] = c01 * id;
  Ji[2][0] = c02 * id;
  Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
  Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
  Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
  Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
  Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
  Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
  *det_out = det;
  return true;
}

int assemble_mesh(MeshGroup& g, std::string& err) {
  const int n = g.n, nt = g.ntet;
  g.V.assign(n, 0.0);
  g.tetV.assign(nt, 0.0);
  std::vector<double> grads(size_t(nt) * 12);
  for (int e = 0; e < nt; ++e) {
    const int32_t* t = &g.tet[4 * e];
    double J[3][3], Ji[3][3], det;
    for (int a = 0; a < 3; ++a) {
      J[a][0] = g.x[t[a + 1]] - g.x[t[0]];
      J[a][1] = g.y[t[a + 1]] - g.y[t[0]];
      J[a][2] = g.z[t[a + 1]] - g.z[t[0]];
    }
    if (!invert3(J, Ji, &det)) {
      err = "degenerate tetrahedron " + std::to_string(e);
      return BPM_EINVAL;
    }
    double* gr = &grads[size_t(e) * 12];
    for (int c = 0; c < 3; ++c) {
      // d phi_a / d x_c = (J^-1)_{c, a-1}
      gr[3 * 1 + c] = Ji[c][0];
      gr[3 * 2 + c] = Ji[c][1];
      gr[3 * 3 + c] = Ji[c][2];
      gr[c] = -(Ji[c][0] + Ji[c][1] + Ji[c][2]);
    }
    g.tetV[e] = std::fabs(det) / 6.0;
    for (int a = 0; a < 4; ++a) g.V[t[a]] += 0.25 * g.tetV[e];
  }
  for (int i = 0; i < n; ++i)
    if (!(g.V[i] > 0.0)) {
      err = "node " + std::to_string(i) + " belongs to no tetrahedron";
      return BPM_EINVAL;
    }

  // pattern: per-row sorted neighbour lists
  std::vector<std::vector<int32_t>> nb(n);
  for (int e = 0; e < nt; ++e)
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) nb[g.tet[4 * e + a]].push_back(g.tet[4 * e + b]);
  g.rowptr.assign(n + 1, 0);
  for (int i = 0; i < n; ++i) {
    auto& v = nb[i];
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
    g.rowptr[i + 1] = g.rowptr[i] + int32_t(v.size());
  }
  g.nnz = g.rowptr[n];
  g.col.resize(g.nnz);
  for (int i = 0; i < n; ++i) std::copy(nb[i].begin(), nb[i].end(), g.col.begin() + g.rowptr[i]);
  auto pos = [&](int i, int j) -> int {
    auto b = g.col.begin() + g.rowptr[i], e = g.col.begin() + g.rowptr[i + 1];
    return int(std::lower_bound(b, e, j) - g.col.begin());
  };
  g.K.assign(g.nnz, 0.0);
  g.D.assign(size_t(g.nnz) * 3, 0.0);
  for (int e = 0; e < nt; ++e) {
    const int32_t* t = &g.tet[4 * e];
    const double* gr = &grads[size_t(e) * 12];
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) {
        int q = pos(t[a], t[b]);
        g.K[q] += g.tetV[e] * (gr[3 * a] * gr[3 * b] + gr[3 * a + 1] * gr[3 * b + 1] + gr[3 * a + 2] * gr[3 * b + 2]);
        for (int c = 0; c < 3; ++c) g.D[3 * size_t(q) + c] += 0.25 * g.tetV[e] * gr[3 * a + c];
      }
  }
  // transposed charge operator on the same (symmetric) pattern: DT(j,k) = D(k,j)
  g.DT.assign(size_t(g.nnz) * 3, 0.0);
  for (int k = 0; k < n; ++k)
    for (int q = g.rowptr[k]; q < g.rowptr[k + 1]; ++q) {
      int j = g.col[q];
      int qt = pos(j, k);
      for (int c = 0; c < 3; ++c) g.DT[3 * size_t(qt) + c] = g.D[3 * size_t(q) + c];
    }

  // interface
  g.partner.assign(n, -1);
  g.aif.assign(n, 0.0);
  for (int p = 0; p < g.nif; ++p) {
    int s = g.iface[2 * p], h = g.iface[2 * p + 1];
    if (s < 0 || s >= n || h < 0 || h >= n || g.layer[s] != 0 || g.layer[h] != 1) {
      err = "interface pair " + std::to_string(p) + " is not (soft node, hard node)";
      return BPM_EINVAL;
    }
    g.partner[s] = h;
    g.partner[h] = s;
  }
  std::vector<double> side_area(n, 0.0);
  for (int e = 0; e < nt; ++e) {
    const int32_t* t = &g.tet[4 * e];
    for (int skip = 0; skip < 4; ++skip) {
      int f[3], k = 0;
      for (int a = 0; a < 4; ++a)
        if (a != skip) f[k++] = t[a];
      bool on = true;
      for (int a = 0; a < 3; ++a) on = on && g.partner[f[a]] >= 0 && g.layer[f[a]] == g.layer[f[0]];
      if (!on) continue;
      double ux = g.x[f[1]] - g.x[f[0]], uy = g.y[f[1]] - g.y[f[0]], uz = g.z[f[1]] - g.z[f[0]];
      double wx = g.x[f[2]] - g.x[f[0]], wy = g.y[f[2]] - g.y[f[0]], wz = g.z[f[2]] - g.z[f[0]];
      double cx = uy * wz - uz * wy, cy = uz * wx - ux * wz, cz = ux * wy - uy * wx;
      double area = 0.5 * std::sqrt(cx * cx + cy * cy + cz * cz);
      for (int a = 0; a < 3; ++a) side_area[f[a]] += area / 3.0;
    }
  }
  // both copies of an interface node use the mean of the two sides' lumped areas
  for (int p = 0; p < g.nif; ++p) {
    int s = g.iface[2 * p], h = g.iface[2 * p + 1];
    double a = 0.5 * (side_area[s] + side_area[h]);
    g.aif[s] = a;
    g.aif[h] = a;
  }

  // node -> tet lists
  g.n2t_ptr.assign(n + 1, 0);
  for (int i = 0; i < 4 * nt; ++i) g.n2t_ptr[g.tet[i] + 1]++;
  for (int i = 0; i < n; ++i) g.n2t_ptr[i + 1] += g.n2t_ptr[i];
  g.n2t.resize(size_t(4) * nt);
  std::vector<int32_t> fill(n, 0);
  for (int e = 0; e < nt; ++e)
    for (int a = 0; a < 4; ++a) {
      int i = g.tet[4 * e + a];
      g.n2t[g.n2t_ptr[i] + fill[i]++] = e;
    }

  double vs = 0.0, c[3] = {0, 0, 0};
  g.vol_layer[0] = g.vol_layer[1] = 0.0;
  for (int i = 0; i < n; ++i) {
    vs += g.V[i];
    c[0] += g.V[i] * g.x[i];
    c[1] += g.V[i] * g.y[i];
    c[2] += g.V[i] * g.z[i];
    g.vol_layer[g.layer[i] ? 1 : 0] += g.V[i];
  }
  for (int k = 0; k < 3; ++k) g.centroid[k] = c[k] / vs;
  return BPM_OK;
}

}  // namespace bpm
