"""FP64 CPU oracle for the TTN trajectory engine -- TEST INFRASTRUCTURE ONLY.

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may
import anything from here.  The GPU engine never calls into this package and
this package never imports the engine; the two share only the op-list input
produced by `workload`.

Contents (each module cites the passage of the paper it follows):
  rng          counter-based uniforms (Philox4x64-10 via numpy's bit generator)
  channels     the SRX / AD channels (Eq. 1-3) and their Pauli twirl (Eq. 9)
  statevector  quantum-trajectory simulation on a dense state vector
               (Sec. III.C; exact Kraus unravelling), lazy ancillas
  densitymatrix exact channel evolution on a dense density matrix
  chp          stabilizer tableau simulator for Clifford + Pauli circuits
  stabrank     Schmidt rank of a stabilizer state across a cut
  closed_forms values the paper's equations fix in closed form
  decoder      final-data lookup decoder and the logical readout
  gradient     exact derivatives of log P(record) by each location's theta
               and gamma (shift rules on the state-vector log P)

Every function is plain, slow and written to be checked against the paper by
eye; precision is float64 / complex128 throughout.
"""
