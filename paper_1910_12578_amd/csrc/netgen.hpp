// Network code generator: turns a reaction-network topology into device code.
//
// The implicit reaction equation of the SDC update (Sec. 2, Eq. 2) is solved
// per zone by Newton with an analytic Jacobian.  For the Jacobian and its LU
// factors to live in registers, every matrix index must be a compile-time
// constant, so the library emits straight-line device functions for the
// network it was initialised with and compiles them at run time.
#pragma once
#include <array>
#include <string>
#include <vector>

namespace sdcgen {

struct Topology {
  int ns = 0;                                 // species
  int nr = 0;                                 // reactions
  std::vector<std::array<int, 2>> reactants;  // [nr] (a, c); c = -1: unimolecular
  std::vector<double> stoich;                 // [nr * ns]
};

// Structural pattern of the Newton matrix I - dt dR/dx and of its LU factors
// in the fixed elimination order (species in index order, energy last).
struct Pattern {
  int n = 0;
  std::vector<int> index;  // [n * n] -> slot in the packed factor array, -1 = structural zero
  int nnz = 0;             // slots, fill-in included
  int nnz_jac = 0;         // slots before fill-in
  long lu_fma = 0;         // multiply-adds of the factorisation
};

// Floating-point operations of the generated functions (add, mul, div, exp and
// log count 1, fused multiply-add counts 2), for the roofline accounting.
struct FlopCount {
  long source = 0;           // net_source: R(x)
  long residual_matrix = 0;  // net_residual_matrix: G and the Newton matrix
  long lu = 0;               // net_lu
  long solve = 0;            // forward and backward substitution
  long exps = 0;             // exp calls per R or residual evaluation
};

FlopCount count_flops(const Topology& t, const Pattern& p);

Pattern build_pattern(const Topology& t);

// Device source (C++ text) defining the network constants and functions
//   net_source, net_residual_matrix<MT>, net_lu_solve<MT>, net_lu<MT>, net_solve_t<MT>,
//   net_residual_dense, net_vjp  (see the generated comments).
std::string generate(const Topology& t, const Pattern& p);

}  // namespace sdcgen
