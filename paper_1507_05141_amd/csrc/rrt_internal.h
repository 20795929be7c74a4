// Internal declarations shared by the library's translation units.
#pragma once
#include <vector>

namespace rrt {

void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w);
void gauss_legendre(int n, double *x, double *w);    // into arrays of n
void real_sh(int lmax, double mu, double phi, double *Y);
// Compton group-to-group tables at nt node temperatures kT (units of the edges; 0 =
// electrons at rest), computed on the GPU in FP64 on the given HIP stream:
// s [nt][G] (cross-section / sigma_T) and p [nt][lmax+1][G][G] (Legendre moments
// p_l^{i->j}); returns a hipError_t value (0 on success)
int compton_tables_gpu(int G, const double *edges, const double *centres, double mec2, int lmax, int nt,
                       const double *kT, std::vector<double> &s, std::vector<double> &p, void *stream);
// the same in a caller's device scratch buffer of compton_scratch_bytes(G, lmax, nt),
// writing s and p to host arrays
size_t compton_scratch_bytes(int G, int lmax, int nt);
int compton_tables_in(int G, const double *edges, const double *centres, double mec2, int lmax, int nt,
                      const double *kT, void *scratch_buf, double *s_out, double *p_out, void *stream);
// the same in the library's static device scratch array (no allocation); returns
// hipErrorInvalidValue when compton_scratch_bytes exceeds compton_static_scratch_bytes()
size_t compton_static_scratch_bytes();
int compton_tables_static(int G, const double *edges, const double *centres, double mec2, int lmax, int nt,
                          const double *kT, double *s_out, double *p_out, void *stream);

}  // namespace rrt
