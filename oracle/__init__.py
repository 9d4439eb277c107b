"""Plain CPU FP64 oracle for the regularised FFT solve of the paper's layered
3D Fredholm equation of the first kind (Leonov & Bakushinsky, arXiv 1703.01216).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only the tests, the smoke check and the benchmark's CPU
baseline leg use it.  It shares no code with the HIP library.

Every routine here is written for a reader checking it against the paper by
eye: plain definitions (direct sums, explicit DFT matrices, dense normal
equations) where the method reaches an exactly defined result, and the
algorithm's steps in order where it iterates.  numpy.fft appears only after
it has been pinned against the explicit DFT of ``oracle.dft``.

Modules
  geometry    grids, the kernel K (Sec. 3, Eq. (8)), sampled offsets, sources, V0
  dft         explicit DFT sums (definition) on small grids
  operator    forward operator: direct quadrature sum and circulant FFT form
  tikhonov    kernel spectrum, spectral Tikhonov estimator, dense Tikhonov
  discrepancy regularisation-parameter choice by the discrepancy principle
  recovery    xi = zeta / V0 and c (Algorithm 1, step 4)
  features    spectral-energy features for the alpha predictor (per kernel-spectrum level)
  mlp         FP64 reference of the alpha-predictor MLP with BF16 emulation
  synth       synthetic data F = A(xi V0) + scaled noise
"""
