// user gate definitions, nested, with parameter expressions (hand-written)
OPENQASM 2.0;
include "qelib1.inc";
gate zzrot(theta) p, q { cx p, q; rz(theta) q; cx p, q; }
gate layer(t, s) x, y, z { ry(t/2) x; zzrot(s*pi) x, y; zzrot(-s) y, z; u3(t, pi/3, -pi/7) z; }
// dup is never applied (a body is only expanded, and checked, on use)
gate dup a, b { layer(0.3, 0.25) a, b, a2dummy; }
qreg q[9];
h q;
layer(0.7, -0.4) q[0], q[4], q[8];
layer(1.1, 0.2) q[1], q[2], q[3];
cu1(pi/8) q[5], q[6];
crz(-0.9) q[6], q[7];
cry(2*sin(pi/6)) q[7], q[0];
ccx q[1], q[5], q[3];
cswap q[8], q[2], q[6];
rzz(0.33) q[2], q[4];
u2(0.1, -0.2) q[5];
sx q[3]; sdg q[1]; t q[0]; tdg q[8];
swap q[0], q[8];
