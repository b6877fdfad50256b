"""FP64 CPU oracle for the sketched-and-truncated polynomial block Krylov method (s-PKSM).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously-correct
reference that the GPU library is checked against.  Only the test suite, the
package's ``smoke()`` check and the benchmark's CPU-baseline leg may import it; the
GPU product path never calls it and shares no code with it.

It follows Palitta, Schweitzer and Simoncini, "Sketched and truncated polynomial
Krylov subspace methods: matrix Sylvester equations" (arXiv 2311.16019):

* ``sketch``      oblivious subspace embeddings (Sec. 2.2): the sparse sign embedding
                  hashed with SplitMix64, the subsampled DCT of Sec. 6, a Gaussian one;
* ``sylvester``   Bartels-Stewart for the small projected equation (Sec. 6 says the
                  small equations are solved that way);
* ``spksm``       Algorithm 1 (s-PKSM) with Prop. 2.1's sketched QR update, the
                  whitened projected equation (eqn:reduced_sk), the residual estimate
                  (eq:resnorm_sk), low-rank factorisation and the two-pass recovery of
                  Sec. 5;
* ``tpksm``       Algorithm 2 (t-PKSM, Appendix A);
* ``full_arnoldi`` the fully orthogonal block Arnoldi Galerkin method (Sec. 2.1), a
                  test reference only;
* ``lowrank``     residual and distance evaluations on low-rank factors;
* ``closed_form`` the sine-transform solution for the 2D Dirichlet Laplacian pair;
* ``adjoint``     gradients of ``tr(P1^T X P2)`` through the transposed equation.

Every numerical readout that the paper leaves open is documented where it is taken.
"""
