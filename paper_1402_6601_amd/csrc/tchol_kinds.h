/* Task kinds of the tile DAGs executed by the persistent kernel.  Included by
   the host planner and by the device code so both number them alike. */
#ifndef TCHOL_KINDS_H
#define TCHOL_KINDS_H
/* factorization (right-looking tile Cholesky) */
#define TK_POTRF 0   /* L_kk = chol(A_kk)                      */
#define TK_TRSM  1   /* A_ik <- A_ik L_kk^{-T},  i > k         */
#define TK_SYRK  2   /* A_ii <- A_ii - L_ik L_ik^T (lower)      */
#define TK_GEMM  3   /* A_ij <- A_ij - L_ik L_jk^T,  i > j > k  */
/* solve L L^T X = B by tiles of rows of B */
#define TK_FTRSV 4   /* Y_k <- L_kk^{-1} B_k                    */
#define TK_FGEMV 5   /* B_i <- B_i - L_ik Y_k,   i > k          */
#define TK_BTRSV 6   /* X_k <- L_kk^{-T} Y_k                    */
#define TK_BGEMV 7   /* Y_i <- Y_i - L_ki^T X_k, i < k          */
/* adjoint of the factorization (reverse tile DAG); P: the adjoint in
   lower-parameter form, Q = P + P^T (twice the symmetric adjoint) */
#define TK_GREV  8   /* Lbar_ik <- Lbar_ik - Q_ij L_jk, i > k, j > k        */
#define TK_TREV  9   /* P_ik = Lbar_ik L_kk^{-1}, i > k                     */
#define TK_DPART 10  /* S_ik = -tril(P_ik^T L_ik), i > k (partial product)   */
#define TK_PREV  11  /* P_kk = the diagonal tile's adjoint                    */
/* mixed precision: the explicit inverse of a diagonal tile, for its solves */
#define TK_TRTRI 12  /* Dinv_k = L_kk^{-1}, DinvT_k = L_kk^{-T} (FP64)        */
/* adjoint: the diagonal tile's partial products, summed by row strips */
#define TK_DRED  13  /* Lbar_kk += sum_i S_ik (i ascending)                  */
/* factorization: two consecutive updates of one tile in one task (K = 2 nb) */
#define TK_GEMM2 14  /* A_ij <- A_ij - L_ik L_jk^T - L_i,k+1 L_j,k+1^T        */
/* adjoint: the diagonal tile's adjoint in closed form (tiles whose order is a
   multiple of 16; others take TK_PREV), three products over TCHOL_PRB x TCHOL_PRB
   blocks, with L_kk^{-T} from TK_TRTRI and Lbar_kk^T (written by TK_DRED into Q_kk) */
#define TK_PADJM 15  /* M_k = Phi(L_kk^T Lbar_kk), lower blocks, stored negated  */
#define TK_PADJY 16  /* Y_k^T = L_kk^{-T} M_k^T, upper blocks                    */
#define TK_PADJS 17  /* Q_kk = L_kk^{-T} Y_k + Y_k^T L_kk^{-1}, Lbar_kk = tril(Q_kk)/2 */
/* adjoint: two consecutive links of a GREV chain in one task (K = 2 nb) */
#define TK_GREV2 18  /* Lbar_ik <- Lbar_ik - Q_ij L_jk - Q_i,j+1 L_j+1,k        */
#define TK_NKINDS 19
#define TCHOL_PRB 64  /* block order of the TK_PADJ* products                      */
#endif
