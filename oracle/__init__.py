"""Reference oracle for the pseudopotential lattice-Boltzmann step with
phase change (Jaramillo, Mapelli, Cabezas-Gomez, "Pseudopotential Lattice
Boltzmann Method for boiling heat transfer: a mesh refinement procedure").

THIS PACKAGE IS TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.
Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import, call or execute anything in it.  The GPU library
never routes through it, and it shares no code with the GPU path.

It is plain serial NumPy in float64 (complex128 also works, which gives
complex-step derivatives for the adjoint checks).  Every function cites
the section / equation of the paper it follows; the places where the
paper is silent or garbled use the readings listed in the module
docstrings (and in the design notes of the repository).

Modules
  lattice  -- D2Q9 velocities, weights, MRT moment matrix (Sec. 2)
  thermo   -- Peng-Robinson EOS, pseudopotential, Maxwell construction,
              latent heat, sigma fit, planar surface tension, kappa rule,
              Stefan similarity constant (Secs. 2, 3, 4.2)
  step     -- one full time step of the method: moments, pseudopotential
              forces, Li source terms, MRT collision, energy equation (RK2),
              streaming with Zou-He walls of either contact-angle model
              (psi-based or modified-psi) and the zero-gradient outflow of
              the 1-D boiling problem (Secs. 2, 4.2)
  adjoint  -- reverse-mode derivative of the step (for the adjoint checks)

Parity status of each function is stated in its module header.
"""
