"""Plain FP64 CPU oracle for the Lyman-alpha mock hot path (arXiv 2310.18996).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call, link or execute anything under this
package; only the tests, the graft smoke check and the CPU-baseline leg of the
benchmark do.  The oracle shares no code with the HIP path: it has its own
Philox, its own Box-Muller, its own power-spectrum table, its own FFTs (numpy)
and its own interpolation, written from the paper and from the published
definitions of the building blocks it cites.

Each module states the passage of the paper it follows (section, equation
label).  Where the paper is silent or ambiguous the reading taken is stated
in the module docstring and in the design notes of the repository.

Modules
-------
philox     Philox4x32-10 counter-based generator and Box-Muller normals.
cosmology  Flat LCDM distance-redshift relation (Table cosmoparams).
power      Analytic P(k), sigma8 normalisation, s(n^2) table (eq:deltaL).
field      k-space modes with Hermitian pairing, delta and eta_par boxes
           (eq:deltaL, eq:eta), by numpy inverse FFT.
lines      Exact evaluation of single z-lines of very large boxes via a plain
           C program (field_lines.c), for full-size sampled parity.
skewers    Ray-march, trilinear interpolation, small-scale field delta_S
           (section "Gaussian fields along lines of sight").
fgpa       g field and the FGPA transform (eq:gfield, eq:FGPA), mean flux
           per redshift bin.
p1d        1D flux power spectrum estimate.
tune       Plain parameter-tuning loop (section "Adjusting mock parameters").
mlp        FP64 multilayer perceptron (forward, backward, Adam) for the
           emulator.
"""
