"""Oracle: the approximant coefficients the paper prints (monomial order a_0..a_4).

TEST INFRASTRUCTURE (see the package docstring).

Table 1 (Section 3.1): fourth-degree minimax polynomials.
  ARCSIN row: 2 asin(tau / sqrt 2) in tau on [0, 1/sqrt 2]  (eps 2.097814e-05)
  ARCCOS row: acos(z) in z on [0, 0.5]                      (eps 1.048949e-05)
  (The intervals are the ones Section 3.1 names for the two pieces.)
Table 2 (Section 3.2): minimax polynomials of exp(-z) on [0, 10], degrees 2-4.
Table 3 (Section 3.2): minimax rational R^4_4 for exp(-z) on [0, 10] (eps 2.227050e-06).
Table 4 (Section 3.3): minimax rational R^4_4 for z ln z on [0.05, 1] (eps 7.342477e-07).
"""

TABLE1_ARCSIN = (2.097797e-05, 1.412840, 1.429881e-02, 6.704361e-02, 6.909677e-02)
TABLE1_ARCSIN_EPS = 2.097814e-05
TABLE1_ARCCOS = (1.570786, -9.990285e-01, -1.429899e-02, -9.481335e-02, -1.381942e-01)
TABLE1_ARCCOS_EPS = 1.048949e-05

TABLE2 = {
    2: ((8.214528e-01, -3.186948e-01, 2.544088e-02), 1.785517e-01),
    3: ((9.174126e-01, -5.631179e-01, 1.015041e-01, -5.519183e-03), 8.259345e-02),
    4: ((9.666313e-01, -7.620584e-01, 2.145386e-01, -2.509526e-02, 1.032877e-03), 3.337085e-02),
}
EXP_CUTOFF = 10.0          # Section 3.2: arguments outside [0, T] give 0, T = 10

TABLE3_NUM = (3.206619e-02, -1.195191e-02, 1.756974e-03, -1.199261e-04, 3.182685e-06)
TABLE3_DEN = (3.206627e-02, 2.011147e-02, 5.853684e-03, 9.780143e-04, 1.251598e-04)
TABLE3_EPS = 2.227050e-06

TABLE4_NUM = (-1.519742e-04, -6.835769e-02, -8.856923e-01, -5.369609e-01, 1.491165)
TABLE4_DEN = (1.532270e-02, 3.987796e-01, 1.461793, 6.827004e-01, -4.469776e-02)
TABLE4_EPS = 7.342477e-07
ENT_CUTOFF = 0.05          # Section 3.3: arguments below T give 0, T = 0.05

KAPPA = 0.33               # Section 3.2: kernel-width scaling factor
