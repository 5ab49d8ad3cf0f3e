/* Internal helpers of the CPU oracle (test infrastructure only; see oracle.h). */
#ifndef FMMKMC_ORACLE_INTERNAL_H
#define FMMKMC_ORACLE_INTERNAL_H

#include "oracle.h"

/* Index-only factors of the three translation operators for one order p,
 * each a (p+1)^2 x (p+1)^2 table indexed [(j,k)][(n,m)]. */
typedef struct or_ops {
    int p, nt;
    cplx *fmm; /* i^{|k|-|m|-|k-m|} A_n^m A_{j-n}^{k-m} / A_j^k          */
    cplx *fml; /* i^{|k-m|-|k|-|m|} A_n^m A_j^k / ((-1)^n A_{j+n}^{m-k}) */
    cplx *fll; /* i^{|m|-|m-k|-|k|} A_{n-j}^{m-k} A_j^k / ((-1)^{n+j} A_n^m) */
} or_ops;

or_ops *or_ops_create(int p);
void or_ops_destroy(or_ops *o);
/* scratch arrays: (p+1)^2 entries, scratch2p: (2p+1)^2 entries */
void ops_p2m_add(const or_ops *o, double q, const double d[3], cplx *M, cplx *scratch);
void ops_m2m(const or_ops *o, const cplx *O, const double Q[3], cplx *M, cplx *scratch);
void ops_m2l_add(const or_ops *o, const cplx *O, const double Q[3], cplx *L, cplx *scratch2p);
void ops_m2l_with_geometry(const or_ops *o, const cplx *O, const cplx *G, cplx *L);
void ops_l2l_add(const or_ops *o, const cplx *O, const double Q[3], cplx *L, cplx *scratch);
void ops_p2l_add(const or_ops *o, double q, const double d[3], cplx *L, cplx *scratch);
double ops_eval_local(const or_ops *o, const cplx *L, const double d[3], cplx *scratch);

#endif
