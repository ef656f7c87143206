/* oracle_internal.h -- shared declarations inside the FP64 oracle (test infrastructure). */
#ifndef CGKS_ORACLE_INTERNAL_H
#define CGKS_ORACLE_INTERNAL_H
#include "cgks_oracle.h"

namespace cgkso {

void solve_dense(int n, double* A, double* b, int nrhs);
void cons_to_prim(const double* Q, double gamma, double prim[5], double* p_out);
double viscosity(const cgkso_params& P, double T);
void time_integrals(double T, double tau, double c[6]);
void point_flux(const cgkso_params& P, double dt, const double* wl, const double* wr, double* out,
                double* dbg);

/* reconstruction (recon.cpp) */
const int NB = 34;       // quartic zero-mean basis, 1 <= |d| <= 4
const int NSTEN = 19;    // cell, 6 face neighbours, 12 edge neighbours
const int NCOL = 75;     // 18 value differences + 19 x 3 normalised gradient components
void stencil_offsets(int off[NSTEN][3]);
const double* recon_operator();  // [NB][NCOL]
void face_gauss_points(double gp[4][2]);
// Reconstruct one variable of one cell; q[19], g[19][3] physical-unit gradients.
// out[6][4][4] = faces (-x,+x,-y,+y,-z,+z) x Gauss points x (value, d/dx, d/dy, d/dz).
// scale: the variable's magnitude squared, for the smoothness floor of the GENO path function
void recon_cell(const cgkso_params& P, const double* q, const double (*g)[3], const double h[3],
                double scale, int mode, double out[6][4][4], double info[4]);
// the same reconstruction evaluated at npts normalised points x: out[n] = (value, d/dx, d/dy, d/dz)
void recon_cell_at(const cgkso_params& P, const double* q, const double (*g)[3], const double h[3],
                   double scale, int mode, int npts, const double (*x)[3], double (*out)[4]);
// the GENO scale of variable v of the conservative state q[5]: rho^2, 2 rho rhoE, (rhoE)^2
double geno_scale(const double* q5, int v);
// GKS-2nd: one variable of one cell from q[7] (cell, -x,+x,-y,+y,-z,+z): face-centre values
// and slopes, out[6][4].
void recon_cell_gks2(const cgkso_params& P, const double* q7, const double h[3], int limited,
                     double out[6][4]);
void recon_cell_gks2_at(const cgkso_params& P, const double* q7, const double h[3], int limited, int npts,
                        const double (*x)[3], double (*out)[4]);

/* MLP (mlp.cpp) */
void mlp_forward(const float* params, const float* x, long n, int bf16, double* logits);

}  // namespace cgkso
#endif
