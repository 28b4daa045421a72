"""FP64 CPU oracle for the FFT eigenstrain / interaction-energy path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import anything in this package.  The
product path (the HIP library and its Python binding) never imports, calls or
links it; the two share no code.

The oracle is a plain, slow, obviously-correct restatement of the method of
Santos-Gueemes, Ortiz and Segurado, "An FFT based approach to account for
elastic interactions in OkMC" (arXiv 2403.09158):

* ``raster``   - defects to eigenstrain fields (Sec. 3.1: loop slab eigenstrain
                 sym(b x n)/e over the extruded loop area; point-defect clusters as
                 dilatations), on the voxel-centre grid of Sec. 3.4.
* ``elastic``  - stiffness tensors and the Green operator built from the inverse
                 acoustic tensor (Sec. 3.2).
* ``solve``    - full-complex FFT solve with the centred frequency labels of
                 Sec. 3.4, then sigma = C:(eps - eps*) (Sec. 3.2).
* ``energy``   - interaction energies from the Betti-reciprocity form (Sec. 2),
                 both brute-force pairwise and the fast exact form.
* ``jumps``    - energy changes of candidate whole-voxel jumps, the biased jump
                 frequencies and the frequency-line selection (Sec. 5 and the
                 OkMC loop of App. B).
* ``okmc``     - one step of the parallel OkMC loop (Sec. 5, App. B): fixed time
                 step, Poisson event counts, one chosen jump per acting defect,
                 energies of the moved list.
* ``dipole``   - the dipole-tensor approximation of the interaction energy
                 (Sec. 2.1).
* ``shift``    - stored defect-type fields translated by the shift theorem
                 (Sec. 3.3, eq. ``shift``) and the energy of the translated
                 defect with a stress field.
* ``dislocation`` - straight dislocation lines by field dislocation mechanics
                 (Sec. 3.1): Nye tensor, incompatible plastic distortion, the
                 Green solve of its symmetric part.

Everything is float64 / complex128 and uses full 3x3 and 3x3x3x3 tensors (no
Voigt shortcuts).  Readings of garbled or silent passages are stated in each
function's docstring.

Parity status: every function here is pinned by a ``-m "not gpu"`` test
against a closed form, an invariant, a brute-force evaluation or a textbook
special case, except the absolute value of anisotropic energies, which only
brute force and invariants pin (the paper's figures carry no numbers).
"""
