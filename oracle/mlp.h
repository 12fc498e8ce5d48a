/* mlp.h -- FP64 per-pair MLP of the oracle (test infrastructure only). */
#ifndef SPINLAT_ORACLE_MLP_H
#define SPINLAT_ORACLE_MLP_H

typedef struct {
    double sigma;    /* RBF width, A */
    double mu_step;  /* RBF spacing, A */
    double sJ, sP;   /* output scales, eV */
    double ex_rc, rc;
} mlp_cfg;

int mlp_nparam(void);
/* out = {J, dJ/dr, phi, dphi/dr} at r */
void mlp_eval(const mlp_cfg *c, const double *p, double r, double out[4]);
/* raw network outputs y = (y0, y1) and dy/dr at r (no cuts, no scales) */
void mlp_raw(const mlp_cfg *c, const double *p, double r, double y[2], double dy[2]);

#endif
