// Internal declarations of the MI355X SD library (not part of the ABI).
#pragma once

#include <cstdint>
#include <cstddef>
#include <string>
#include <vector>

#include "../../include/chorus.h"

namespace chorus {

constexpr int kMaxOrder = 6;

// 1D SD operators of order N (Section 3): solution points xs (Chebyshev-Gauss),
// flux points xf (0, Legendre-Gauss, 1), interpolation I[m][s] = h_s(xf[m]),
// flux-polynomial derivative D[s][m] = l_m'(xs[s]) and quadrature weights.
struct Basis1D {
    int N = 0;
    double xs[kMaxOrder] = {};
    double xf[kMaxOrder + 1] = {};
    double I[kMaxOrder + 1][kMaxOrder] = {};
    double D[kMaxOrder][kMaxOrder + 1] = {};
    double w[kMaxOrder] = {};
};
bool build_basis(int N, Basis1D &b);

// Face-neighbour record of one element face.
struct FaceLink {
    int32_t nbr_elem = -1;  // -1 on boundary faces
    int32_t nbr_face = -1;
    int32_t orient = -1;    // swap*4 + flip1*2 + flip2
    int32_t bc = -1;        // face tag
};

// Byte offsets of the arrays inside the device geometry image.
struct DeviceLayout {
    size_t solgeo = 0;     // f64 [E][13][NP]: G[3 d][3 c] = |J| grad xi_d / |J|, 1/|J|, x/r^3
    size_t fluxgeo = 0;    // f64 [E][3 d][3 c][NFL]: |J| grad xi_d at d-flux points
    size_t link = 0;       // i32 [E][6]: neighbour element or -1
    size_t info = 0;       // i32 [E][6]: nbr_face | orient << 3 | (bc + 1) << 6
    size_t solw = 0;       // f64 [E][NP]: w w w |J|
    size_t solgeo32 = 0;   // f32 copy of solgeo (mixed mode)
    size_t fluxgeo32 = 0;  // f32 copy of fluxgeo (mixed mode)
    size_t xsol = 0;       // f64 [E][3][NP]: solution-point coordinates
    size_t rflux = 0;      // f64 [E][3 d][NFL]: radius at the d-flux points
    size_t rflux32 = 0;    // f32 copy of rflux (mixed mode)
    size_t total = 0;
};

struct Mesh {
    int N = 0;
    int64_t E = 0;
    std::vector<double> xyz;        // [n_nodes][3]
    std::vector<int64_t> elem20;    // [E][20]
    std::vector<int32_t> face_bc;   // [E][6]
    std::vector<int64_t> match_id;  // [n_nodes]
    Basis1D basis;
    std::vector<FaceLink> links;    // [E][6]
    // host geometry (FP64)
    std::vector<double> xsol;       // [E][NP][3]
    std::vector<double> jac;        // [E][NP]
    std::vector<double> met;        // [E][NP][3][3]
    std::vector<double> metf;       // [E][3][NFL][3]  (interface ends made antisymmetric)
    std::vector<double> rflux;      // [E][3][NFL] radius at the d-flux points
    double rflux_min = 0.0, rflux_max = 0.0;
    int64_t n_faces = 0, n_wall_faces = 0;
    DeviceLayout layout;
    std::vector<unsigned char> image;  // host copy of the device image
    void *dev_image = nullptr;          // registered caller-owned device buffer
    int device = -1;
    // mixed-mode background registered by chorus_set_background
    bool bg_ready = false;
    const void *bg_ws = nullptr;
    chorus_physics bg_phys{};
    int64_t n_nodes() const { return (int64_t)xyz.size() / 3; }
};

// Builders (host).  Return CHORUS_OK or an error code and set the message.
int build_shell(const chorus_shell_desc &d, Mesh &m);
int build_from_hex20(const chorus_hex20_desc &d, Mesh &m);
int finish_mesh(Mesh &m);  // faces, geometry, device image

void set_error(const std::string &msg);

}  // namespace chorus
