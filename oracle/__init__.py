"""CPU oracle for the sliced sparse-state contraction (Pan, Chen & Zhang, arXiv:2111.03011).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check of the package entry
file and the CPU-baseline leg of the benchmark may import or run anything in this
package.  The library's compute path never calls it and shares no code with it: the
oracle builds its own gates, its own tensor network and its own contraction path from
the circuit description, in plain numpy complex128.

What it computes (paper, "Method" and Appendix A/B):
  psi_hat_Sigma(s) = sum over slices sigma in Sigma of <s| U_sigma |0^n>,
where U_sigma is the circuit's network with every sliced bond fixed to the value that
sigma assigns it.  With Sigma the full set this is the exact amplitude <s|U|0^n>
(Appendix B.2, slicing).  Two independent routes compute it:
  * statevector.simulate  - gate-by-gate state vector, slicing as inserted projectors;
  * contract.sparse_amplitudes - pairwise tensordot contraction of the network, one
    group and one slice at a time.
sampling.py draws bitstrings by |psi_hat|^2 (main text, sampling paragraph) and
metrics.py holds the error, fidelity, XEB and efficiency formulas.

Pins (tests/test_oracle_*.py): closed forms of the gate set and Eq. (1), brute-force
Kronecker products on 1-3 qubits, norm 1, the two routes agreeing, slice sums equal to
unsliced results, path independence, the Appendix A worked example, the SplitMix64
published output sequence and the Table I identities.
"""
