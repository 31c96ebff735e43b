"""Amortized interval subdivision on MI355X (gfx950).

Moroz, "Sparse Tensors and Subdivision Methods for Finding the Zero Set of
Polynomial Equations", arXiv 2406.09857: interval evaluation of a polynomial
system on the live boxes of one level of a bisection tree, stored as a
Compressed Sparse Fiber tree, by Horner partial evaluation one variable per
CSF depth (Algorithm 2), followed by the exclusion filter and bisection of
Algorithm 3.

The arithmetic runs in hand-written HIP kernels behind the C-ABI library
``libvoxcsf.so``; :mod:`.binding` marshals torch tensors to it.  Importing the
package does not load the library; the first call does, and fails loudly if
it has not been built.
"""
