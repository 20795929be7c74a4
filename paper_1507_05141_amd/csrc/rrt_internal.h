// Internal declarations shared by the library's translation units.
#pragma once
#include <vector>

namespace rrt {

void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w);
void real_sh(int lmax, double mu, double phi, double *Y);
void compton_tables(int G, const double *edges, const double *centres, double mec2, int lmax,
                    std::vector<double> &s, std::vector<double> &A, std::vector<double> &p);

}  // namespace rrt
