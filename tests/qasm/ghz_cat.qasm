// GHZ preparation on a 7-qubit register, then a cat-state chain on a second
// register; barriers between the parts (hand-written test input)
OPENQASM 2.0;
include "qelib1.inc";
qreg a[7];
qreg b[5];
creg c[12];
h a[0];
cx a[0],a[1];
cx a[1],a[2];
cx a[2],a[3];
cx a[3],a[4];
cx a[4],a[5];
cx a[5],a[6];
barrier a;
h b[0];
cx b[0],b[1]; cx b[1],b[2]; cx b[2],b[3]; cx b[3],b[4];
barrier a, b;
measure a -> c[0];
