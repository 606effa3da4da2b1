/*
 * lbm_ref.h -- the CPU oracle for the D2Q37 thermal lattice Boltzmann step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this library: only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant
 * generator with the GPU library.
 *
 * Plain serial FP64 C, written for reading, not for speed.  Every function
 * follows the definitions of the paper (Calore, Gabbana, Schifano,
 * Tripiccione, "Optimization of Lattice Boltzmann Simulations on Heterogeneous
 * Computers", arXiv:1703.04594), section 3 ("Lattice Boltzmann methods"):
 *   - the BGK evolution equation, eq. (1);
 *   - the macroscopic moments rho, rho*u, D*rho*T, eq. (2);
 *   - the pull form of the update, eq. (4): gather then compute;
 *   - the per-step order propagate -> bc -> collide (section 5, the
 *     heterogeneous control flow).
 * Where the paper defers to its model references (velocity labels, weights,
 * equilibrium, wall rule) the readings are stated at each function.
 *
 * Layout of every population array handed across this interface:
 * canonical [37][lx][ly], y fastest, FP64.  Field arrays are [lx][ly].
 */
#ifndef LBM_REF_H
#define LBM_REF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define REF_NPOP 37

/* Boundary kinds.  x is periodic or open; each y side is a wall, open, or
 * (both sides together) periodic.  "Open" means: a pull whose source lies
 * outside the lattice yields NaN and nothing overwrites it.  Open sides exist
 * only so that a window cut out of a larger lattice can be evolved: after n
 * steps the sites farther than 3n from an open side are exact. */
enum { REF_WALL = 0, REF_PERIODIC = 1, REF_OPEN = 2 };

typedef struct ref_lattice ref_lattice;

/* Canonical population order and lattice constants (see lbm_ref.c). */
void   ref_velocity_table(int32_t ex[REF_NPOP], int32_t ey[REF_NPOP]);
double ref_scale_c(void);
void   ref_weights(double w[REF_NPOP]);
/* Residual of the 9 quadrature moment equations in quad precision, as doubles. */
void   ref_quadrature_residuals(double res[9]);

/* Equilibrium f^eq_l(rho, u, T) for all l (expanded Hermite form). */
void   ref_feq(double rho, double ux, double uy, double T, double out[REF_NPOP]);

/* Returns NULL on invalid arguments (tau <= 0.5, lx or ly < 1, bad kinds). */
ref_lattice* ref_create(int32_t lx, int32_t ly, int32_t xbc, int32_t ybc_bottom,
                        int32_t ybc_top, double tau, double g_y,
                        double t_bottom, double t_top);
void   ref_destroy(ref_lattice* L);

/* All return 0 on success, nonzero on a state error. */
int    ref_init(ref_lattice* L, const double* rho, const double* ux,
                const double* uy, const double* T);
int    ref_set_pops(ref_lattice* L, const double* src);
int    ref_get_pops(const ref_lattice* L, double* dst);
int    ref_propagate(ref_lattice* L);
int    ref_bc(ref_lattice* L);
int    ref_collide(ref_lattice* L);
int    ref_step(ref_lattice* L, int64_t n);
int    ref_get_macros(const ref_lattice* L, double* rho, double* ux,
                      double* uy, double* T);
int    ref_conservation(const ref_lattice* L, double out[4]);
/* Threads the build uses (1 unless compiled with OpenMP). */
int    ref_threads(void);

#ifdef __cplusplus
}
#endif
#endif
