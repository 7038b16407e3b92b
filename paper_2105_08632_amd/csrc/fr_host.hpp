// Host-side set-up of the HIP path: reference operators per (element type,
// degree) and per-element geometry.  Runs once per context; nothing here is
// on the timed path.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace frh {

enum { QUAD = 0, TRI = 1, HEX = 2, TET = 3, PRI = 4 };

struct RefOps {
  int type = -1, p = 0, nd = 0, ns = 0, nf = 0, nface = 0, nfp = 0, nvert = 0;
  int wl = 0, wc = 0;                 // compressed row widths
  std::vector<double> sp, fp;         // reference solution / flux points
  std::vector<double> nref;           // [nf][nd]
  std::vector<int> fface;             // [nf]
  std::vector<int> face_off;          // [nface + 1] first flux point of each face
  std::vector<double> M0, D, Cor;     // [nf][ns], [nd][ns][ns], [ns][nf]
  std::vector<double> Dc, G;          // [nd][ns][ns]
  std::vector<int> m0c, dcc, gc, crc, ddc; // compressed rows
  std::vector<double> m0v, dcv, gv, crv, ddv;
  std::vector<double> wsol;           // quadrature weights at solution points
  // 1-D factors of tensor elements (n1 = p + 1): derivative matrix, lifting
  // h+-_i = l_i(+-1)/w_i and end values l_i(+-1)
  std::vector<double> D1, hp, hm, lp, lm;
  std::vector<std::vector<int>> face_verts;
  // scheme: 0 FR-DG, 1 FR-SDRT, 2 SDRT (tensor elements)
  int scheme = 0;
  // SDRT lines: interior SD flux points z_1..z_p of a line, sdI[j][i] =
  // l_i(z_{j+1}) (solution points to interior flux points), sdD[i][j] =
  // psi_j'(x_i) (derivative of the flux-point Lagrange basis psi_0..psi_{p+1}
  // at the solution points), sdend[(d * nl + l) * 2 + side] = the external
  // flux point at the -1 (side 0) / +1 (side 1) end of line l along axis d
  std::vector<double> sdz, sdI, sdD;
  std::vector<int> sdend;
};

// Builds the FR-DG reference operators.  beta enters G (self gradient).
// tri_pts: [ns][2] triangle points (triangles' solution points, the
// triangular faces of tetrahedra and prisms, the prisms' cross-section);
// tet_pts: [ns][3] solution points of tetrahedra.  Either may be null where
// unused.
bool build_ref(int type, int p, double beta, int scheme, const double* tri_pts, const double* tet_pts, RefOps& out,
               std::string& err);

// SDRT: row d of detJ J^{-1} at the interior flux points of every line along
// axis d, [ne][nd][nl][p][nd] (nl = lines per axis).
void build_sd_metric(const RefOps& R, int nd, int64_t ne, const double* xyz, int max_vert, std::vector<double>& Sint);

struct Geometry {
  int nd = 0, ns = 0, nf = 0, nface = 0;
  int64_t ne = 0;
  std::vector<double> S, Jinv, rdet, nrm, magN;   // per element, element-major
  std::vector<int> nbfp, nbr;
  std::vector<int> nbface, back;      // [ne][nface], [ne][nface][nfp]
  std::vector<double> Sint;           // SDRT: see build_sd_metric (empty otherwise)
};

// Metric terms at solution / flux points and the flux-point pairing across
// faces, found by matching physical positions relative to the face centroid.
bool build_geometry(const RefOps& ref, int nd, int64_t ne, const double* xyz, int max_vert, const int64_t* nbr,
                    const int8_t* nbr_face, int max_face, Geometry& g, std::string& err);

// Cross-type face data of one element group of a mixed mesh.
struct MixInfo {
  std::vector<int> nbpt;              // [ne_g][nf]: the paired point's local index in the neighbour
  std::vector<int> nbt;               // [ne_g][nface]: 1 when the neighbour is of the other type
  std::vector<int64_t> nbg;           // [ne_g][nface]: the neighbour's mesh index
};

// The same over ngrp contiguous groups of one element type each (elements
// gstart[g] .. gstart[g+1]-1; refs indexed by element type).  Each group's
// arrays are group-local; nbfp holds the partner's index in a flux-point
// numbering that runs over the groups in order, minus the group's first
// point (so a kernel given the group's slice of a shared trace array reads
// partners in other groups at negative or past-the-end offsets).  mix (may
// be null) receives the cross-type data per group.
bool build_geometry_groups(const RefOps* const* refs, int nd, int64_t ne, const int8_t* etype, const double* xyz,
                           int max_vert, const int64_t* nbr, const int8_t* nbr_face, int max_face, int ngrp,
                           const int64_t* gstart, Geometry* g, MixInfo* mix, std::string& err);

// Checks the truncated viscous Jacobian's assumptions: distinct face
// neighbours and a second face layer that does not fold back onto the first.
bool check_stencil(int64_t ne, int nface, const int* nbr, std::string& err);

}  // namespace frh
