// Host-side FP64 gate construction (see host_gates.cpp).
#pragma once
#include <vector>

struct TnModelHost {
    int L = 0;
    std::vector<double> h_bond;     // (L-1) * 16 complex, interleaved
    std::vector<int> jump_site;
    std::vector<double> jump_op;    // njump * 4 complex, interleaved
    std::vector<double> gamma;
};

std::vector<double> build_bond_gate(int kind, const TnModelHost& m, int b, double tau);
std::vector<double> embed_purified(const std::vector<double>& g4, int dkl, int dkr);
