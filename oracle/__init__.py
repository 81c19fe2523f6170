"""FP64 CPU oracle of rank-constrained SCM estimation (Kubo et al., APSIPA 2019).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in this
package.  The GPU library never calls it, and it shares no code with the GPU
path (it never imports ``paper_1908_01964_amd``).

Contents (each module cites the passage it follows):

* ``naive``      - the literal EM/MAP iteration, E-step eqs. (13)-(16) and
                   M-step eqs. (17)-(20), with one M x M inverse per bin.
* ``accel``      - the second-stage accelerated iteration (Algorithm 2,
                   eqs. (46)-(56)), scalar-only per bin.
* ``first_stage``- the first-stage accelerated iteration (Algorithm 1).
* ``objective``  - negative log-posterior / log-likelihood of the model
                   (eqs. (2)-(10)), by slogdet + solve.
* ``bruteforce`` - E-step by generic Gaussian conditioning and M-step by
                   numerical maximisation of the Q function (eq. (12)).
* ``extract``    - multichannel Wiener filter: posterior mean of s given x.
* ``adjoint_ref``- FP64 torch (CPU) autograd of the accelerated forward, and
                   central finite differences of the numpy forward.

Everything is float64 / complex128.
"""
