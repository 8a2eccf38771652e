// Host-side one-dimensional operator tables (long double, rounded to double).
#pragma once

#include <vector>

namespace dgfv {

std::vector<long double> lgl_nodes(int N);
std::vector<long double> lgl_weights(int N);
std::vector<long double> ld_D(int N);               // (N+1)^2, unrounded
std::vector<long double> ld_interp(int N, int M);   // (M+1) x (N+1), unrounded

std::vector<double> op_nodes(int N);
std::vector<double> op_weights(int N);
std::vector<double> op_D(int N);                    // (N+1)^2
std::vector<double> op_vleg_inv(int N);             // (N+1)^2
std::vector<double> op_interp(int N, int M);        // (M+1) x (N+1)
std::vector<double> op_project(int M, int N);       // (N+1) x (M+1), M > N
std::vector<double> op_dg2fv(int N, int NFV);       // NFV x (N+1)
std::vector<double> op_fv2dg(int N, int NFV);       // (N+1) x NFV
std::vector<double> op_face_interp(int N, int NFV); // (NFV+1) x (N+1)
// mortars (Section 3.2.3): half k = 0 ([-1, 0]) or 1 ([0, 1]) of a big side of degree N
std::vector<double> op_mortar_interp(int N, int k);   // (N+1) x (N+1): big side -> nodes of half k
std::vector<double> op_mortar_project(int N, int k);  // (N+1) x (N+1): half k's flux -> big side
// their sub-cell variants on N_FV equal sub-faces per direction, by overlap
std::vector<double> op_mortar_fv_interp(int NFV, int k);   // NFV x NFV: big side -> sub-faces of half k (means)
std::vector<double> op_mortar_fv_project(int NFV, int k);  // NFV x NFV: half k's sub-face fluxes -> big side

}  // namespace dgfv
