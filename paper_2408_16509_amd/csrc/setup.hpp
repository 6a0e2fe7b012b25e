// Host-side setup of the FR right-hand side: element operators, mesh connectivity
// and geometry, ready to upload.  Plain C++17, no device code.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace frmi {

constexpr int kHex = 0;
constexpr int kTet = 1;
constexpr int kPyr = 2;
constexpr int kMaxP = 4;

// One-dimensional operators of hexahedra of order p (Gauss--Legendre points).
struct HexOps {
  int p = 0, n1 = 0, nsp = 0, nfp = 0, nfpf = 0;
  double x[kMaxP + 1] = {}, w[kMaxP + 1] = {};
  double lm[kMaxP + 1] = {}, lp[kMaxP + 1] = {};   // l_a(-1), l_a(+1)
  double D[kMaxP + 1][kMaxP + 1] = {};             // D[a][b] = l_b'(x_a)
  double Dh[kMaxP + 1][kMaxP + 1] = {};            // D - gR' lp^T - gL' lm^T (correction folded in)
  double cp[kMaxP + 1] = {}, cm[kMaxP + 1] = {};   // gR'(x_a), -gL'(x_a)
  double Vm[kMaxP + 1][kMaxP + 1] = {};            // 1-D orthonormal Legendre Vandermonde V[a][m]
  double Vmi[kMaxP + 1][kMaxP + 1] = {};           // its inverse
};

// Operators of the order-4 tetrahedron (alpha-optimised points of Fig. mesh).
struct TetOps {
  static constexpr int nsp = 35, nfp = 60, nfpf = 15;
  double pts[nsp][3];
  int fp_src[nfp];                 // solution point collocated with each flux point
  int fp_face[nfp];
  double nref[4][3];               // unit outward reference normals
  double D[3][nsp][nsp];           // D[i][z][n] = d l_n / d xi_i at x_z
  double lift[nsp][nfp];           // DG lifting M^{-1} E
  double Dh[3][nsp][nsp];          // D_i - lift * (n~_i at the collocated flux points): the
                                   // normal trace of f~ folded into the derivative
  double weights[nsp];             // integral of l_z
  double V[nsp][nsp];              // orthonormal modal basis at the points, V[z][m]
  double Vinv[nsp][nsp];
  int deg[nsp];                    // total degree of mode m
};

// Operators of the order-4 pyramid with an affine base (reference base [-1,1]^2 at
// z = -1, apex (0,0,1)).  Space: the rational pyramid space of dimension 55 spanned by
// (x/s)^i (y/s)^j s^max(i,j) z^c, s = (1 - z)/2, c <= 4 - max(i,j); it holds P_4, and
// its trace is Q_4 on the base and P_4 on the triangles.  Solution points: 5 layers at
// the Gauss--Legendre z nodes, layer k the (5-k)^2 Gauss--Legendre grid scaled by s
// (x fastest).  Flux points: the base's 5 x 5 Gauss--Legendre grid (x fastest), then
// each triangle (corners c0 c1 c2) the 15 face points of the tetrahedron's face in
// barycentric coordinates.  Correction: the DG lifting M^{-1} E.
struct PyrOps {
  static constexpr int nsp = 55, nfp = 85, nfaces = 5;
  double pts[nsp][3];
  double fpts[nfp][3];
  int fp_face[nfp];
  int face_off[nfaces + 1];        // flux points of face f: face_off[f] .. face_off[f+1]-1
  double nref[nfaces][3];          // unit outward reference normals
  double interp[nfp][nsp];         // l_j at the flux points
  double D[3][nsp][nsp];           // D[i][z][j] = d l_j / d xi_i at x_z
  double lift[nsp][nfp];           // DG lifting M^{-1} E
};

// A block of elements of one type, in the native (element-fastest) layout.
struct Block {
  int etype = kHex;
  int64_t n = 0, e_pad = 0;
  int nsp = 0, nfp = 0, nfaces = 0, nfpf = 0;
  std::vector<int64_t> elems;      // global element ids in native order
  std::vector<int32_t> canon_pos;  // native index -> canonical index (input order within the type)
  int ngeo = 0;
  std::vector<double> geo;         // [ngeo][e_pad]
  std::vector<int32_t> nbr_elem;   // [nfaces][e_pad] neighbour's local index (same block)
  std::vector<int32_t> nbr_info;   // [nfaces][e_pad] nbr_face | orient << 3 | is_left << 12
  std::vector<double> sol_xyz;     // [n][nsp][3] physical solution points (canonical order)
  // Curved elements: stored metric terms (empty for straight elements), rows of e_pad
  // values.  Hexahedra: S row d at solution point pt (row pt*9 + d*3 + j, S = J G^{-1}),
  // 1/J at solution point pt (row 9 nsp + pt), and at flux point fp of face 2d+s row d
  // of S (row 10 nsp + fp*3 + j).  Tetrahedra (flux points are solution points): S at
  // solution point pt (row pt*10 + 3i + j) and J (row pt*10 + 9), then the scaled normal
  // S^T n~ at flux point fp (row 10 nsp + fp*3 + j).
  std::vector<double> cmet;
};

struct Setup {
  HexOps hex;
  TetOps tet;
  PyrOps pyr;
  std::vector<Block> blocks;
  int n_orient = 0;
  std::vector<int32_t> orient_perm;  // [n_orient][max face points]
  int perm_stride = 0;
};

// Builders.  Return an empty string on success, else an error message; `code`
// receives 1 for argument errors, 2 for mesh errors, 3 for unsupported options.
void build_hex_ops(int p, HexOps& ops);
void build_tet_ops(TetOps& ops);
void build_pyr_ops(const TetOps& tet, PyrOps& ops);   // tet: its face points are the triangles
std::string build_setup(int order, int64_t n_vert, const double* xyz, const double* period,
                        int64_t n_elem, const int32_t* etype, const int64_t* enodes,
                        int e_align, int elem_order, Setup& out, int& code);

// Metric terms of curved hexahedra of geometry order q (the hexahedral block of `s`,
// built by build_setup from the elements' corners).  ho: [n_elem][(q+1)^3] node
// indices in tensor order (node i + (q+1)(j + (q+1)k) at reference point
// (-1 + 2i/q, -1 + 2j/q, -1 + 2k/q)).  metric 0: conservative (curl) form, 1: cross
// product.  Fills Block::cmet and replaces Block::sol_xyz with the curved points.
std::string build_curved_hex(int q, int metric, const double* xyz, const int64_t* ho, Setup& s, int& code);

// The same for curved tetrahedra of geometry order q (1..4; the tetrahedral block of
// `s`).  ho: [n_elem][(q+1)(q+2)(q+3)/6] node indices, nodes (i, j, k) with
// i + j + k <= q, k outermost, then j, then i, at (-1 + 2i/q, -1 + 2j/q, -1 + 2k/q).
std::string build_curved_tet(int q, int metric, const double* xyz, const int64_t* ho, Setup& s, int& code);

}  // namespace frmi
