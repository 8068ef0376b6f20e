function mpc = case5_handmade
% Small meshed test case written for the MATPOWER reader tests (hand-made
% numbers, not taken from any published case): non-contiguous bus numbers,
% a reference bus that is not first, two generators on one bus, an
% out-of-service generator and branch, a transformer with tap and phase
% shift, an unlimited branch, a bus shunt, quadratic and linear costs.
mpc.version = '2';

%% system MVA base
mpc.baseMVA = 100;

%% bus data
%	bus_i	type	Pd	Qd	Gs	Bs	area	Vm	Va	baseKV	zone	Vmax	Vmin
mpc.bus = [
	10	1	40	12	0	0	1	1	0	230	1	1.06	0.94;
	20	3	0	0	0	0	1	1	0	230	1	1.06	0.94;
	30	2	25	8	0	5	1	1	0	230	1	1.06	0.94;
	40	1	30	9	1	0	1	1	0	230	1	1.06	0.94;
	50	1	20	6	0	0	1	1	0	230	1	1.06	0.94;
];

%% generator data
%	bus	Pg	Qg	Qmax	Qmin	Vg	mBase	status	Pmax	Pmin
mpc.gen = [
	20	0	0	150	-150	1	100	1	200	0;
	30	0	0	60	-60	1	100	1	80	0;
	30	0	0	40	-40	1	100	1	50	0;
	50	0	0	30	-30	1	100	0	40	0;
];

%% branch data
%	fbus	tbus	r	x	b	rateA	rateB	rateC	ratio	angle	status	angmin	angmax
mpc.branch = [
	20	10	0.01	0.06	0.03	250	250	250	0	0	1	-360	360;
	20	30	0.02	0.08	0.02	150	150	150	0	0	1	-360	360;
	10	40	0.015	0.07	0.02	0	0	0	0	0	1	-360	360;
	30	40	0.01	0.05	0.01	120	120	120	0.98	2	1	-360	360;
	40	50	0.02	0.09	0.02	100	100	100	0	0	1	-360	360;
	10	50	0.03	0.1	0.01	90	90	90	0	0	0	-360	360;
	30	50	0.025	0.08	0.02	110	110	110	0	0	1	-360	360;
];

%% generator cost data
%	2	startup	shutdown	n	c(n-1)	...	c0
mpc.gencost = [
	2	0	0	3	0.02	20	0;
	2	0	0	3	0.05	15	0;
	2	0	0	2	30	0	0;
	2	0	0	3	0.04	25	0;
];
